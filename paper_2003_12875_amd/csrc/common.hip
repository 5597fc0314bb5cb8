// common.hip -- model-independent kernels: dataset validation, the tile
// schedule of the batched pass (sets of events, or one dataset at many
// parameter points), and the read-out of a batched fit.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "reduce.h"

namespace nllmi {

// Work items of the batched pass.  The events [0, n) are cut into chunks
// (ChunkGrid: K rounds of G chunks, chunk j = r G + b streamed by block b;
// chunks of C events, the last round's G equal shares of what remains), and
// an item is the part of one set inside one chunk.  Every block streams the
// same number of events, and at any time the grid reads neighbouring
// chunks (one contiguous range per block reads HBM ~10 % slower).  Items
// are numbered in event order, so the items of a set are consecutive
// (tile_off[s] .. tile_off[s+1]) and so are those of a chunk
// (chunk_first[j] .. chunk_first[j+1]).  An empty set gets one empty item,
// in the chunk that holds its offset.  The offsets must be non-decreasing
// within [0, n]; if any is not, every set of the batch is flagged (status
// NLL_ERR_ARG) and gets one empty item.  At most n_sets + G K items.
// floor(a / b) for 0 <= a < 2^53 (exact as a double), b > 0: the
// double-precision quotient is off by at most one and is corrected with
// integer products; a 64-bit integer division is a long software routine
// here.
__device__ __forceinline__ int64_t div_floor(int64_t a, int64_t b) {
  int64_t q = (int64_t)((double)a / (double)b);
  const int64_t r = a - q * b;
  if (r < 0) --q;
  else if (r >= b) ++q;
  return q;
}

__device__ __forceinline__ int64_t chunk_start(int64_t j, const ChunkGrid& g) {
  const int64_t full = (int64_t)(g.K - 1) * g.G;
  if (j <= full) return j * g.C;
  return g.base + div_floor((j - full) * g.L, g.G);
}
// the chunk that holds event e (0 <= e < n)
__device__ __forceinline__ int64_t chunk_of(int64_t e, const ChunkGrid& g) {
  if (e < g.base) return div_floor(e, g.C);
  return (int64_t)(g.K - 1) * g.G + div_floor((e - g.base + 1) * g.G - 1, g.L);
}
// the chunks [j0, j1] of set s's items
__device__ inline void set_chunks(const int64_t* __restrict__ offsets, int s, int n_sets, const ChunkGrid& g,
                                  int flag, int64_t& j0, int64_t& j1) {
  const int64_t nc = (int64_t)g.G * g.K;
  const int64_t a = flag ? 0 : offsets[s], e = flag ? 0 : offsets[s + 1];
  if (flag || g.n == 0) {
    j0 = j1 = (int64_t)s * nc / n_sets;  // empty items spread over the chunks, in order
  } else if (e == a) {
    j0 = j1 = a < g.n ? chunk_of(a, g) : nc - 1;
  } else {
    j0 = chunk_of(a, g);
    j1 = chunk_of(e - 1, g);
  }
}

constexpr int kSchedThreads = 1024;  // one block: the per-set counts and their prefix

__global__ __launch_bounds__(kSchedThreads) void k_schedule(const int64_t* __restrict__ offsets, int n_sets,
                                                     const ChunkGrid g, int64_t* __restrict__ tile_off,
                                                     int* __restrict__ set_flag,
                                                     int64_t* __restrict__ chunk_first) {
  __shared__ int64_t scan[kSchedThreads];
  __shared__ int any_bad;
  const int t = threadIdx.x;
  if (t == 0) any_bad = 0;
  __syncthreads();
  const int per = (n_sets + kSchedThreads - 1) / kSchedThreads;
  const int s0 = min(n_sets, t * per), s1 = min(n_sets, s0 + per);
  for (int s = s0; s < s1; ++s) {
    const int64_t a = offsets[s], b = offsets[s + 1];
    if (!(a >= 0 && b >= a && b <= g.n)) atomicOr(&any_bad, 1);
  }
  __syncthreads();
  const int bad = any_bad;
  int64_t local = 0;
  for (int s = s0; s < s1; ++s) {
    set_flag[s] = bad;
    int64_t j0, j1;
    set_chunks(offsets, s, n_sets, g, bad, j0, j1);
    local += j1 - j0 + 1;
  }
  scan[t] = local;
  __syncthreads();
  for (int d = 1; d < kSchedThreads; d <<= 1) {
    const int64_t v = t >= d ? scan[t - d] : 0;
    __syncthreads();
    scan[t] += v;
    __syncthreads();
  }
  int64_t run = scan[t] - local;  // exclusive prefix
  for (int s = s0; s < s1; ++s) {
    tile_off[s] = run;
    int64_t j0, j1;
    set_chunks(offsets, s, n_sets, g, bad, j0, j1);
    run += j1 - j0 + 1;
  }
  if (t == kSchedThreads - 1) tile_off[n_sets] = scan[kSchedThreads - 1];
  if (n_sets == 0)
    for (int64_t j = t; j <= (int64_t)g.G * g.K; j += kSchedThreads) chunk_first[j] = 0;
}

// The items of every set (one thread per set), and chunk_first: the first
// item of each chunk (chunk_first[G K] = the item count).
__global__ __launch_bounds__(kBlock) void k_items(const int64_t* __restrict__ offsets, int n_sets, const ChunkGrid g,
                                                  const int64_t* __restrict__ tile_off,
                                                  const int* __restrict__ set_flag, WorkItem* __restrict__ items,
                                                  int64_t* __restrict__ chunk_first) {
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= n_sets) return;
  const int flag = set_flag[s];
  const int64_t a = flag ? 0 : offsets[s], e = flag ? 0 : offsets[s + 1];
  int64_t j0, j1;
  set_chunks(offsets, s, n_sets, g, flag, j0, j1);
  int64_t prev = -1;  // the chunk of the previous set's last item
  if (s > 0) {
    int64_t p0, p1;
    set_chunks(offsets, s - 1, n_sets, g, set_flag[s - 1], p0, p1);
    prev = p1;
  }
  const int64_t i0 = tile_off[s];
  for (int64_t j = prev + 1; j <= j0; ++j) chunk_first[j] = i0;
  for (int64_t j = j0; j <= j1; ++j) {
    const int64_t i = i0 + (j - j0);
    if (j > j0) chunk_first[j] = i;
    int64_t lo = a, hi = e;
    if (e > a) {
      const int64_t r0 = chunk_start(j, g), r1 = chunk_start(j + 1, g);
      lo = a > r0 ? a : r0;
      hi = e < r1 ? e : r1;
    }
    items[i] = WorkItem{lo, hi, s, flag};
  }
  if (s == n_sets - 1)
    for (int64_t j = j1 + 1; j <= (int64_t)g.G * g.K; ++j) chunk_first[j] = tile_off[n_sets];
}

__global__ __launch_bounds__(kBlock) void k_fit_final(int n_sets, int P, GDState gd, double* theta_out,
                                                     double* nll_out, double* grad_out,
                                                     int* status_out) {
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= n_sets) return;
  for (int q = 0; q < P; ++q) {
    theta_out[(size_t)s * P + q] = gd.th_acc[(size_t)s * P + q];
    if (grad_out) grad_out[(size_t)s * P + q] = gd.g_acc[(size_t)s * P + q];
  }
  const double f = gd.f_acc[s];
  if (nll_out) nll_out[s] = f;
  if (status_out) status_out[s] = __builtin_isfinite(f) ? 0 : gd.last_status[s];
}

__global__ __launch_bounds__(kBlock) void k_check_range(const double* __restrict__ x, int64_t n,
                                                       double lo, double hi,
                                                       unsigned long long* __restrict__ bad) {
  unsigned long long local = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const double v = x[i];
    local += !(v >= lo && v <= hi);
  }
  if (local) atomicAdd(bad, local);
}

hipError_t launch_schedule(const int64_t* offsets, int n_sets, const ChunkGrid& g, int64_t* tile_off,
                           int* set_flag, WorkItem* items, int64_t* chunk_first, hipStream_t st) {
  hipLaunchKernelGGL(k_schedule, dim3(1), dim3(kSchedThreads), 0, st, offsets, n_sets, g, tile_off, set_flag,
                     chunk_first);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n_sets <= 0) return e;
  hipLaunchKernelGGL(k_items, dim3((n_sets + kBlock - 1) / kBlock), dim3(kBlock), 0, st, offsets, n_sets, g,
                     tile_off, set_flag, items, chunk_first);
  return hipGetLastError();
}

// Points mode: every set is the whole dataset [0, n), evaluated at its own
// parameter point.  Virtual offsets s * n give each set its event count n
// (the finishing kernel's n_s); ceil(n / tile) items per set, or one empty
// item if n == 0; no flags; one round of G chunks, the blocks taking equal
// runs of consecutive items.  One thread per item (and per set for the
// per-set arrays, per block for chunk_first).
__global__ __launch_bounds__(kBlock) void k_points(int n_sets, int64_t n, int64_t tile, int64_t per, int G,
                                                   int64_t* __restrict__ offsets, int64_t* __restrict__ tile_off,
                                                   int* __restrict__ set_flag, WorkItem* __restrict__ items,
                                                   int64_t* __restrict__ chunk_first) {
  const int64_t total = (int64_t)n_sets * per;
  for (int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x; b <= G; b += (int64_t)gridDim.x * kBlock)
    chunk_first[b] = b * total / G;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
    const int64_t s = i / per, k = i - s * per;
    const int64_t start = k * tile;
    items[i] = WorkItem{start < n ? start : n, start + tile < n ? start + tile : n, (int32_t)s, 0};
  }
  for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s <= n_sets; s += (int64_t)gridDim.x * kBlock) {
    offsets[s] = s * n;
    tile_off[s] = s * per;
    if (s < n_sets) set_flag[s] = 0;
  }
}

hipError_t launch_points(int n_sets, int64_t n, int64_t tile, int G, int64_t* offsets, int64_t* tile_off,
                         int* set_flag, WorkItem* items, int64_t* chunk_first, hipStream_t st) {
  const int64_t per = n > 0 ? (n + tile - 1) / tile : 1;
  int64_t blocks = ((int64_t)n_sets * per + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_points, dim3((unsigned)blocks), dim3(kBlock), 0, st, n_sets, n, tile, per, G, offsets,
                     tile_off, set_flag, items, chunk_first);
  return hipGetLastError();
}

hipError_t launch_fit_final(int n_sets, int P, const GDState& gd, double* theta_out, double* nll_out,
                            double* grad_out, int* status_out, hipStream_t st) {
  const int grid = (n_sets + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_fit_final, dim3(grid > 0 ? grid : 1), dim3(kBlock), 0, st, n_sets, P, gd, theta_out,
                     nll_out, grad_out, status_out);
  return hipGetLastError();
}

// Sum of the per-event weights: each thread a double-double sum over a
// fixed stride, the block's hi and lo parts summed by block_sum_vals, one
// partial per block; then one block adds the partials in block order.
__global__ __launch_bounds__(kBlock) void k_wsum_part(const double* __restrict__ w, int64_t n, DD* __restrict__ part) {
  __shared__ double buf[2 * (kBlock + 1)];
  __shared__ DD tot[2];
  DD acc{0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) acc = dd_add1(acc, w[i]);
  const double v[2] = {acc.hi, acc.lo};
  block_sum_vals<2, kBlock>(v, buf, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = dd_add(tot[0], tot[1]);
}

__global__ __launch_bounds__(kBlock) void k_wsum_final(const DD* __restrict__ part, int n_part, double* __restrict__ out) {
  __shared__ DD tot[1];
  RecordSum<1, kBlock> rs;
  rs.issue(part, n_part);
  rs.reduce(part, n_part, tot);
  if (threadIdx.x == 0) *out = tot[0].hi + tot[0].lo;
}

hipError_t launch_wsum(const double* w, int64_t n, double* part, double* out, hipStream_t st) {
  int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > kWsumBlocks) blocks = kWsumBlocks;
  if (blocks < 1) blocks = 1;
  DD* p = reinterpret_cast<DD*>(part);
  hipLaunchKernelGGL(k_wsum_part, dim3((unsigned)blocks), dim3(kBlock), 0, st, w, n, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_wsum_final, dim3(1), dim3(kBlock), 0, st, p, (int)blocks, out);
  return hipGetLastError();
}

hipError_t launch_check_range(const double* x, int64_t n, double lo, double hi, unsigned long long* bad,
                              hipStream_t st) {
  int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_check_range, dim3((unsigned)blocks), dim3(kBlock), 0, st, x, n, lo, hi, bad);
  return hipGetLastError();
}

// Read-bandwidth probe: streams n doubles once with the streaming kernels'
// access pattern and load policy but no arithmetic (tiles of 8 x 256
// consecutive doubles, round robin over a persistent grid, loads two tiles
// ahead, non-temporal) and writes one sum per block, so that the loads
// cannot be dropped.  Measures the HBM read rate a streaming kernel can
// reach on this device, the yardstick next to the data sheet's peak.
__global__ __launch_bounds__(kBlock) void k_read_probe(const double* __restrict__ x, int64_t n,
                                                      double* __restrict__ out) {
  constexpr int U = 8;
  const int64_t tile = (int64_t)kBlock * U, ntile = n / tile, G = gridDim.x;
  auto ld = [&](int64_t t, int u) -> double {
    return t < ntile ? __builtin_nontemporal_load(&x[t * tile + (int64_t)u * kBlock + threadIdx.x]) : 0.0;
  };
  double acc = 0.0;
  double r0[U], r1[U], r2[U];
  int64_t tl = blockIdx.x;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    r0[u] = ld(tl, u);
    r1[u] = ld(tl + G, u);
  }
  for (; tl < ntile; tl += G) {
#pragma unroll
    for (int u = 0; u < U; ++u) r2[u] = ld(tl + 2 * G, u);
#pragma unroll
    for (int u = 0; u < U; ++u) acc += r0[u];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      r0[u] = r1[u];
      r1[u] = r2[u];
    }
  }
  for (int64_t i = ntile * tile + (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += G * kBlock) acc += x[i];
  __shared__ double s[kBlock];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = s[0];
}

hipError_t launch_read_probe(const double* x, int64_t n, double* out, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_read_probe, dim3((unsigned)blocks), dim3(kBlock), 0, st, x, n, out);
  return hipGetLastError();
}

}  // namespace nllmi
