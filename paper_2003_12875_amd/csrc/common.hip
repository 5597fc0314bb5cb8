// common.hip -- model-independent kernels: dataset validation, the tile
// schedule of the batched pass (sets of events, or one dataset at many
// parameter points), and the read-out of a batched fit.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "reduce.h"

namespace nllmi {

// Item counts per set and their exclusive prefix.  The offsets must be
// non-decreasing within [0, n_total]; if any is not, every set of the batch
// is flagged (status NLL_ERR_ARG) and gets one empty item, so the number of
// items never exceeds n_total / tile + n_sets.
__global__ __launch_bounds__(kBlock) void k_schedule(const int64_t* __restrict__ offsets, int n_sets,
                                                     int64_t n_total, int64_t tile,
                                                     int64_t* __restrict__ tile_off,
                                                     int* __restrict__ set_flag) {
  __shared__ int64_t scan[kBlock];
  __shared__ int any_bad;
  const int t = threadIdx.x;
  if (t == 0) any_bad = 0;
  __syncthreads();
  const int per = (n_sets + kBlock - 1) / kBlock;
  const int s0 = min(n_sets, t * per), s1 = min(n_sets, s0 + per);
  for (int s = s0; s < s1; ++s) {
    const int64_t a = offsets[s], b = offsets[s + 1];
    if (!(a >= 0 && b >= a && b <= n_total)) atomicOr(&any_bad, 1);
  }
  __syncthreads();
  const int bad = any_bad;
  int64_t local = 0;
  for (int s = s0; s < s1; ++s) {
    set_flag[s] = bad;
    const int64_t len = bad ? 0 : offsets[s + 1] - offsets[s];
    local += len > 0 ? (len + tile - 1) / tile : 1;
  }
  scan[t] = local;
  __syncthreads();
  for (int d = 1; d < kBlock; d <<= 1) {
    const int64_t v = t >= d ? scan[t - d] : 0;
    __syncthreads();
    scan[t] += v;
    __syncthreads();
  }
  int64_t run = scan[t] - local;  // exclusive prefix
  for (int s = s0; s < s1; ++s) {
    tile_off[s] = run;
    const int64_t len = bad ? 0 : offsets[s + 1] - offsets[s];
    run += len > 0 ? (len + tile - 1) / tile : 1;
  }
  if (t == kBlock - 1) tile_off[n_sets] = scan[kBlock - 1];
}

// The work items of every set (one thread per set), in tile_off order: the
// batched kernel then reads an item's set and range with one load instead
// of searching the prefix.
__global__ __launch_bounds__(kBlock) void k_items(const int64_t* __restrict__ offsets, int n_sets, int64_t tile,
                                                  const int64_t* __restrict__ tile_off,
                                                  const int* __restrict__ set_flag, WorkItem* __restrict__ items) {
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= n_sets) return;
  const int flag = set_flag[s];
  const int64_t a = flag ? 0 : offsets[s], b = flag ? 0 : offsets[s + 1];
  const int64_t i0 = tile_off[s], i1 = tile_off[s + 1];
  for (int64_t i = i0; i < i1; ++i) {
    const int64_t start = a + (i - i0) * tile;
    items[i] = WorkItem{start, start + tile < b ? start + tile : b, s, flag};
  }
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

hipError_t launch_schedule(const int64_t* offsets, int n_sets, int64_t n_total, int64_t tile,
                           int64_t* tile_off, int* set_flag, WorkItem* items, hipStream_t st) {
  hipLaunchKernelGGL(k_schedule, dim3(1), dim3(kBlock), 0, st, offsets, n_sets, n_total, tile, tile_off, set_flag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n_sets <= 0) return e;
  hipLaunchKernelGGL(k_items, dim3((n_sets + kBlock - 1) / kBlock), dim3(kBlock), 0, st, offsets, n_sets, tile,
                     tile_off, set_flag, items);
  return hipGetLastError();
}

// Points mode: every set is the whole dataset [0, n), evaluated at its own
// parameter point.  Virtual offsets s * n give each set its event count n
// (the finishing kernel's n_s); ceil(n / tile) items per set, or one empty
// item if n == 0; no flags.  One thread per item (and per set for the
// per-set arrays).
__global__ __launch_bounds__(kBlock) void k_points(int n_sets, int64_t n, int64_t tile, int64_t per,
                                                   int64_t* __restrict__ offsets, int64_t* __restrict__ tile_off,
                                                   int* __restrict__ set_flag, WorkItem* __restrict__ items) {
  const int64_t total = (int64_t)n_sets * per;
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

hipError_t launch_points(int n_sets, int64_t n, int64_t tile, int64_t* offsets, int64_t* tile_off, int* set_flag,
                         WorkItem* items, hipStream_t st) {
  const int64_t per = n > 0 ? (n + tile - 1) / tile : 1;
  int64_t blocks = ((int64_t)n_sets * per + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_points, dim3((unsigned)blocks), dim3(kBlock), 0, st, n_sets, n, tile, per, offsets, tile_off,
                     set_flag, items);
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
