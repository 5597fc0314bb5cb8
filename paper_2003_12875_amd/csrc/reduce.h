// reduce.h -- compensated, deterministic reductions (wave64 -> LDS -> grid).
//
// Per-thread sums are plain FP64; from the block level up values travel as
// double-double pairs (hi, lo).  Addition is Knuth's TwoSum of the high
// parts plus the low parts, renormalised; it is exactly commutative, so the
// xor-butterfly leaves every lane with the same bits and the result does not
// depend on scheduling.  Across blocks the partial sums
// are written by each block and combined in block order by a following
// kernel (the kernel boundary makes them visible across the chip's XCDs).
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

namespace nllmi {

struct DD {
  double hi, lo;
};

__device__ inline DD dd_add(DD x, DD y) {
  const double s = x.hi + y.hi;
  const double bb = s - x.hi;
  const double err = (x.hi - (s - bb)) + (y.hi - bb);
  const double t = err + (x.lo + y.lo);
  const double h = s + t;
  return DD{h, t - (h - s)};
}

// double-double plus double (TwoSum of the high parts, then renormalise)
__device__ inline DD dd_add1(DD x, double y) {
  const double s = x.hi + y;
  const double bb = s - x.hi;
  const double err = (x.hi - (s - bb)) + (y - bb);
  const double t = err + x.lo;
  const double h = s + t;
  return DD{h, t - (h - s)};
}

template <int N>
constexpr int pow2_floor() {
  int p = 1;
  while (2 * p <= N) p *= 2;
  return p;
}

// lanes per accumulator when NV accumulators share `threads` lanes (at most
// one wave, so that a group never straddles two waves)
template <int NV, int THREADS>
constexpr int lanes_per_acc() {
  constexpr int s = pow2_floor<(THREADS / NV > 0 ? THREADS / NV : 1)>();
  return s > 64 ? 64 : s;
}

// xor-butterfly over aligned groups of W lanes (W a power of two <= 64); a
// double-double sum is exactly commutative, so every lane of a group ends
// with the same bits.
template <int W>
__device__ inline DD group_sum_dd(DD v) {
#pragma unroll
  for (int off = W / 2; off >= 1; off >>= 1) {
    const DD o{__shfl_xor(v.hi, off, 64), __shfl_xor(v.lo, off, 64)};
    v = dd_add(v, o);
  }
  return v;
}

// Block sum (BLOCK threads) of NV plain per-thread values into NV
// double-double totals out[] (LDS; visible to every thread on return).
// The values are transposed through buf (NV * (BLOCK + 1) doubles): value j
// is summed by S lanes (S = lanes_per_acc), lane k adding entries k, k + S,
// ... in order (compensated), then by an xor-butterfly over the S lanes.
// The order depends only on NV and BLOCK: results are reproducible.
template <int NV, int BLOCK>
__device__ inline void block_sum_vals(const double (&v)[NV], double* buf, DD* out) {
  constexpr int S = lanes_per_acc<NV, BLOCK>();
  constexpr int PER = BLOCK / S;
  constexpr int LD = BLOCK + 1;  // row stride: rows start in different banks
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < NV; ++j) buf[j * LD + t] = v[j];
  __syncthreads();
  const int j = t / S, k = t % S;
  DD acc{0.0, 0.0};
  if (j < NV) {
    double x[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) x[m] = buf[j * LD + k + m * S];
    acc.hi = x[0];
#pragma unroll
    for (int m = 1; m < PER; ++m) acc = dd_add1(acc, x[m]);
  }
  acc = group_sum_dd<S>(acc);
  if (j < NV && k == 0) out[j] = acc;
  __syncthreads();
}

// A record for a lane that may have none: lanes with `in` false read a
// zero record instead, so that every lane issues the load with neither a
// branch nor a select after it (a select would wait for the load at once,
// and a branch hides it from the waits that follow).  Both pointers are
// taken as global memory: a generic pointer would make this a flat load,
// which the LDS waits would then count too.
static __device__ const DD g_zero_record = {0.0, 0.0};
typedef const double __attribute__((address_space(1))) gdouble;
__device__ __forceinline__ DD load_record(const DD* src, int64_t i, bool in) {
  const gdouble* p = in ? (const gdouble*)(src + i) : (const gdouble*)&g_zero_record;
  return DD{p[0], p[1]};
}

// Fixed-order sum of `count` records of NV double-double values (record r
// at src[r * NV], written by an earlier kernel) by one block of BLOCK
// threads, in two phases so that callers can issue their other loads
// between them: issue() starts the loads of the first B records of every
// lane, reduce() adds them (and any further batches) and combines lanes.
// Accumulator j is served by the S consecutive threads [j S, (j+1) S): lane
// k sums records k, k + S, ... in order, then the S lanes (one wave at
// most) are combined by an xor-butterfly.  The order depends only on count
// and NV, so results are reproducible.  The totals land in out[NV].  B:
// records per lane in flight (one memory round trip covers S * B records).
template <int NV, int BLOCK, int B_ = 8>
struct RecordSum {
  // at most one wave per accumulator: no cross-wave step (a barrier and an
  // LDS round trip cost more than the longer per-lane chains)
  static constexpr int S0 = pow2_floor<(BLOCK / NV > 0 ? BLOCK / NV : 1)>();
  static constexpr int S = S0 > 64 ? 64 : S0;
  static constexpr int B = B_;
  static_assert(S * NV <= BLOCK, "lanes per accumulator");
  DD buf[B];

  __device__ void issue(const DD* src, int64_t count) {
    const int t = threadIdx.x;
    const int j = t / S, k = t % S;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int64_t r = k + (int64_t)b * S;
      buf[b] = load_record(src, r * NV + j, j < NV && r < count);
    }
  }

  __device__ void reduce(const DD* src, int64_t count, DD* out) {
    const int t = threadIdx.x;
    const int j = t / S, k = t % S;
    DD acc = buf[0];
#pragma unroll
    for (int b = 1; b < B; ++b) acc = dd_add(acc, buf[b]);
    for (int64_t r0 = k + (int64_t)B * S; r0 < count; r0 += (int64_t)B * S) {
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int64_t r = r0 + (int64_t)b * S;
        buf[b] = load_record(src, r * NV + j, j < NV && r < count);
      }
#pragma unroll
      for (int b = 0; b < B; ++b) acc = dd_add(acc, buf[b]);
    }
    acc = group_sum_dd<S>(acc);
    if (j < NV && k == 0) out[j] = acc;
    __syncthreads();
  }
};

// The same sum over records stored value-major (value j of record r at
// src[j * count + r]: the S lanes of an accumulator read consecutive
// addresses), with each lane's batch of B records added as a pairwise tree
// (a dependent chain of log2 B additions instead of B - 1).  The order
// depends only on count and NV.
template <int NV, int BLOCK, int B_ = 8>
struct RecordSumT {
  static constexpr int S0 = pow2_floor<(BLOCK / NV > 0 ? BLOCK / NV : 1)>();
  static constexpr int S = S0 > 64 ? 64 : S0;
  static constexpr int B = B_;
  static_assert(S * NV <= BLOCK, "lanes per accumulator");
  static_assert((B & (B - 1)) == 0, "batch: a power of two");
  DD buf[B];
  __device__ void load(const DD* src, int64_t count, int64_t r0) {
    const int t = threadIdx.x;
    const int j = t / S, k = t % S;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int64_t r = r0 + k + (int64_t)b * S;
      buf[b] = load_record(src, (int64_t)j * count + r, j < NV && r < count);
    }
  }
  __device__ DD tree() {
#pragma unroll
    for (int w = 1; w < B; w *= 2)
#pragma unroll
      for (int b = 0; b + w < B; b += 2 * w) buf[b] = dd_add(buf[b], buf[b + w]);
    return buf[0];
  }
  __device__ void issue(const DD* src, int64_t count) { load(src, count, 0); }
  __device__ void reduce(const DD* src, int64_t count, DD* out) {
    const int t = threadIdx.x;
    const int j = t / S, k = t % S;
    DD acc = tree();
    for (int64_t r0 = (int64_t)B * S; r0 < count; r0 += (int64_t)B * S) {
      load(src, count, r0);
      acc = dd_add(acc, tree());
    }
    acc = group_sum_dd<S>(acc);
    if (j < NV && k == 0) out[j] = acc;
    __syncthreads();
  }
};

__device__ inline int block_sum_int(int v, int* lds) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  v = lds[0] + lds[1] + lds[2] + lds[3];
  __syncthreads();
  return v;
}

}  // namespace nllmi
