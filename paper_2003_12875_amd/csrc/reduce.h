// reduce.h -- compensated, deterministic reductions (wave64 -> LDS -> grid).
//
// Values travel as double-double pairs (hi, lo).  Addition is Knuth's
// TwoSum of the high parts plus the low parts, renormalised; it is exactly
// commutative, so the xor-butterfly leaves every lane with the same bits and
// the result does not depend on scheduling.  Across blocks the partial sums
// are combined by the last block to finish, in block order.
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

// Cross-block visibility of partial sums (other XCDs included): stores are
// followed by an agent-scope release fence before the ticket increment; the
// finishing block issues an acquire fence before reading.
__device__ inline void store_dd(DD* p, DD v) {
  __hip_atomic_store(&p->hi, v.hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&p->lo, v.lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline DD load_dd(const DD* p) {
  return DD{__hip_atomic_load(&p->hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
            __hip_atomic_load(&p->lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)};
}

}  // namespace nllmi
