// reduce.h -- compensated, deterministic reductions (wave64 -> LDS -> grid).
//
// Values travel as double-double pairs (hi, lo).  Addition is Knuth's
// TwoSum of the high parts plus the low parts, renormalised; it is exactly
// commutative, so the xor-butterfly leaves every lane with the same bits and
// the result does not depend on scheduling.  Across blocks the partial sums
// are written by each block and combined in block order by a following
// kernel (the kernel boundary makes them visible across the chip's XCDs).
#pragma once

#include <hip/hip_runtime.h>

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

// Sum of NV double-double values over the 64 lanes of a wave (all lanes
// receive the result).
template <int NV>
__device__ inline void wave_sum_dd(DD (&v)[NV]) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      DD o{__shfl_xor(v[j].hi, off, 64), __shfl_xor(v[j].lo, off, 64)};
      v[j] = dd_add(v[j], o);
    }
  }
}

// Sum over the block (256 threads = 4 waves).  The NV totals land in out[]
// (LDS), visible to every thread on return; thread j combines accumulator j
// so that no thread holds the 4 * NV wave partials at once.
// lds must hold 4 * NV DD values.
template <int NV>
__device__ inline void block_sum_dd(DD (&v)[NV], DD* lds, DD* out) {
  wave_sum_dd<NV>(v);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) lds[wave * NV + j] = v[j];
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    const int j = threadIdx.x;
    out[j] = dd_add(dd_add(lds[j], lds[NV + j]), dd_add(lds[2 * NV + j], lds[3 * NV + j]));
  }
  __syncthreads();
}

// Fixed-order sum of `count` records of NV double-double values (record r
// at src[r * NV], written by an earlier kernel) by one block of BLOCK
// threads.  Accumulator j is served by the S consecutive threads
// [j S, (j+1) S), S the largest power of two <= BLOCK / NV: lane k sums
// records k, k + S, ... in order (four loads in flight), then the S lanes
// are combined by a fixed xor-butterfly (and, for S > 64, the waves in
// order through lds[BLOCK / 64]).  The order depends only on count and NV,
// so results are reproducible.  The totals land in out[NV].
template <int NV, int BLOCK>
__device__ inline void sum_records(const DD* src, int64_t count, DD* lds, DD* out) {
  constexpr int S0 = BLOCK / NV;
  constexpr int S = S0 >= 512 ? 512 : S0 >= 256 ? 256 : S0 >= 128 ? 128 : S0 >= 64 ? 64 : S0 >= 32 ? 32
                  : S0 >= 16 ? 16 : S0 >= 8 ? 8 : S0 >= 4 ? 4 : S0 >= 2 ? 2 : 1;
  static_assert(S >= 1 && S * NV <= BLOCK, "lanes per accumulator");
  const int t = threadIdx.x;
  const int j = t / S, k = t % S;
  DD acc{0.0, 0.0};
  if (j < NV) {
    int64_t r = k;
    for (; r + 3 * S < count; r += 4 * S) {
      const DD a0 = src[r * NV + j];
      const DD a1 = src[(r + S) * NV + j];
      const DD a2 = src[(r + 2 * S) * NV + j];
      const DD a3 = src[(r + 3 * S) * NV + j];
      acc = dd_add(dd_add(dd_add(dd_add(acc, a0), a1), a2), a3);
    }
    for (; r < count; r += S) acc = dd_add(acc, src[r * NV + j]);
  }
  constexpr int W = S < 64 ? S : 64;
#pragma unroll
  for (int off = W / 2; off >= 1; off >>= 1) {
    DD o{__shfl_xor(acc.hi, off, 64), __shfl_xor(acc.lo, off, 64)};
    acc = dd_add(acc, o);
  }
  if constexpr (S <= 64) {
    if (j < NV && k == 0) out[j] = acc;
  } else {
    if ((t & 63) == 0) lds[t >> 6] = acc;
    __syncthreads();
    if (t < NV) {
      DD v = lds[t * (S / 64)];
      for (int q = 1; q < S / 64; ++q) v = dd_add(v, lds[t * (S / 64) + q]);
      out[t] = v;
    }
  }
  __syncthreads();
}

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
