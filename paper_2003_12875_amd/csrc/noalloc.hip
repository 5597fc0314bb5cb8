// noalloc.hip -- the batched evaluation without allocation: every scratch
// buffer of the pass lives in one fixed device array per GPU, so that the
// call never allocates device memory (for callers under HIP graph capture
// or in loops that must not allocate).
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "kernels.h"
#include "nll.h"
#include "runtime.h"

using namespace nllmi;

namespace {

// The array itself.  Host code never passes its name to a kernel or a copy
// (on the host the name is only a stand-in): the device address comes from
// hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[NLL_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
std::map<int, unsigned char*> g_addr;  // device ordinal -> address of that device's copy

// the device's copy of the array; the caller has made `device` current
nll_status scratch_on(int device, unsigned char** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_addr.find(device);
  if (it != g_addr.end()) {
    *out = it->second;
    return NLL_OK;
  }
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return NLL_ERR_DEVICE;
  g_addr[device] = static_cast<unsigned char*>(p);
  *out = static_cast<unsigned char*>(p);
  return NLL_OK;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

extern "C" nll_status nll_eval_batched_noalloc(nll_model* m, int32_t n_sets, const int64_t* offsets,
                                               const double* theta, double* nll_out, double* grad_out,
                                               int32_t* status_out) {
  nll_status st = batched_args_ok(m, n_sets, offsets, theta, nll_out);
  if (st != NLL_OK || n_sets == 0) return st;
  // layout: item prefix | set flags | work items | chunks' first items |
  // per-set constants | per-set tables (models with them) | item records
  const size_t items = (size_t)batched_items_bound(m, n_sets);
  const size_t chunks = items - (size_t)n_sets - 1;
  const size_t o_flag = align256(((size_t)n_sets + 1) * sizeof(int64_t));
  const size_t o_items = o_flag + align256((size_t)n_sets * sizeof(int));
  const size_t o_first = o_items + align256(items * sizeof(WorkItem));
  const size_t o_consts = o_first + align256((chunks + 1) * sizeof(int64_t));
  const size_t o_aux = o_consts + align256((size_t)n_sets * sizeof(PerTheta));
  const size_t o_part = o_aux + (m->ops->aux ? align256((size_t)n_sets * kAuxWords * sizeof(double)) : 0);
  const size_t need = o_part + items * batched_record_bytes(m);
  if (need > (size_t)NLL_NOALLOC_SCRATCH_BYTES) return NLL_ERR_SCRATCH;
  DeviceGuard guard(m->device);
  unsigned char* base = nullptr;
  if ((st = scratch_on(m->device, &base)) != NLL_OK) return st;
  SetsScratch s;
  s.tile_off = reinterpret_cast<int64_t*>(base);
  s.set_flag = reinterpret_cast<int*>(base + o_flag);
  s.items = reinterpret_cast<WorkItem*>(base + o_items);
  s.chunk_first = reinterpret_cast<int64_t*>(base + o_first);
  s.consts = reinterpret_cast<PerTheta*>(base + o_consts);
  s.aux = m->ops->aux ? reinterpret_cast<double*>(base + o_aux) : nullptr;
  s.partials = reinterpret_cast<double*>(base + o_part);
  return eval_batched_on(m, n_sets, offsets, theta, nll_out, grad_out, status_out, s);
}
