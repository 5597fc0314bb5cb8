// host_jit.cpp -- the C ABI of the just-in-time densities: the density
// expression is pasted into the device source of jit_source.h, compiled
// with hipRTC for the model's device, loaded as a code object, and its four
// kernels are launched through the module API.
#include <hip/hip_runtime_api.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "jit_source.h"
#include "kernels.h"
#include "nll.h"
#include "runtime.h"

using namespace nllmi;

namespace {

constexpr int kJitMaxParams = 8;  // MAXP of the device source
constexpr int kJitThreads = 256;  // NTH of the device source
constexpr int kJitBlocksPerCu = 4;  // stream blocks per CU at most (fewer where fewer fit)

// mirrors JitArgs of the device source (same member types and order)
struct JitArgsHost {
  const double* x;
  long long n;
  const double* theta;
  double* nll_out;
  double* grad_out;
  double* partials;
  int* status;
  const double* glx;
  const double* glw;
  double lo, hi;
  double par_lo[kJitMaxParams], par_hi[kJitMaxParams];
  int par_free[kJitMaxParams];
  int n_blocks;
};

}  // namespace

struct nll_jit_model {
  int device = 0;
  hipStream_t stream = nullptr;
  int n_cu = 256;
  int n_param = 0;
  double lo = 0.0, hi = 0.0;
  double par_lo[kJitMaxParams] = {}, par_hi[kJitMaxParams] = {};
  int par_free[kJitMaxParams] = {};
  hipModule_t module = nullptr;
  hipFunction_t f_stream[2] = {}, f_finish[2] = {};  // [0] NLL alone, [1] with gradient
  int stream_blocks_per_cu[2] = {1, 1};               // resident at once, so the grid is one wave of blocks
  const double* x = nullptr;
  int64_t n = -1;
  double* partials = nullptr;
  int* status = nullptr;
  unsigned long long* dbad = nullptr;
  double* glx = nullptr;
  double* glw = nullptr;
};

namespace {

void copy_log(const std::string& s, char* log, int32_t cap) {
  if (!log || cap <= 0) return;
  const size_t n = std::min<size_t>(s.size(), (size_t)cap - 1);
  std::memcpy(log, s.data(), n);
  log[n] = '\0';
}

// compile the device source for the model's device; code object into out
nll_status compile(const std::string& src, int device, std::vector<char>& out, std::string& log) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return NLL_ERR_DEVICE;
  std::string arch = std::string("--offload-arch=") + prop.gcnArchName;
  const size_t colon = arch.find(':');  // feature suffixes (e.g. ":sramecc+:xnack-") stay off
  if (colon != std::string::npos) arch.resize(colon);
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "nll_jit.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
    return NLL_ERR_DEVICE;
  const char* opts[] = {arch.c_str(), "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
  const hiprtcResult r = hiprtcCompileProgram(prog, 7, opts);
  size_t ls = 0;
  hiprtcGetProgramLogSize(prog, &ls);
  log.assign(ls, '\0');
  if (ls) hiprtcGetProgramLog(prog, &log[0]);
  if (r != HIPRTC_SUCCESS) {
    hiprtcDestroyProgram(&prog);
    return NLL_ERR_ARG;
  }
  size_t cs = 0;
  hiprtcGetCodeSize(prog, &cs);
  out.resize(cs);
  hiprtcGetCode(prog, out.data());
  hiprtcDestroyProgram(&prog);
  return NLL_OK;
}

template <class T>
nll_status jit_alloc(T** p, size_t count) {
  *p = nullptr;
  const hipError_t e = hipMalloc(reinterpret_cast<void**>(p), (count ? count : 1) * sizeof(T));
  if (e == hipSuccess) return NLL_OK;
  return e == hipErrorOutOfMemory ? NLL_ERR_OOM : NLL_ERR_DEVICE;
}

template <class T>
void jit_free(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

}  // namespace

extern "C" {

nll_status nll_jit_create(const nll_jit_desc* d, nll_jit_model** out, char* log, int32_t log_cap) {
  copy_log("", log, log_cap);
  if (!d || !out || !d->density || !d->param_lo || !d->param_hi) return NLL_ERR_ARG;
  *out = nullptr;
  if (d->n_param < 1 || !(d->obs_lo < d->obs_hi)) return NLL_ERR_ARG;
  if (d->n_param > kJitMaxParams || std::strlen(d->density) > 4096) return NLL_ERR_UNSUPPORTED;
  for (int k = 0; k < d->n_param; ++k)
    if (!(d->param_lo[k] <= d->param_hi[k])) return NLL_ERR_ARG;
  std::string src = jit_source_template();
  const size_t dual_at = src.find("@DUAL@");
  if (dual_at != std::string::npos) src.replace(dual_at, 6, jit_dual_source());
  const std::string expr = d->density;
  for (size_t at = src.find("@EXPR@"); at != std::string::npos; at = src.find("@EXPR@", at + expr.size()))
    src.replace(at, 6, expr);
  src = "#define NP " + std::to_string(d->n_param) + "\n" + src;
  DeviceGuard guard(d->device);
  std::vector<char> code;
  std::string clog;
  nll_status st = compile(src, d->device, code, clog);
  copy_log(clog, log, log_cap);
  if (st != NLL_OK) return st;
  nll_jit_model* m = new (std::nothrow) nll_jit_model();
  if (!m) return NLL_ERR_OOM;
  m->device = d->device;
  m->stream = reinterpret_cast<hipStream_t>(d->stream);
  m->n_param = d->n_param;
  m->lo = d->obs_lo;
  m->hi = d->obs_hi;
  for (int k = 0; k < d->n_param; ++k) {
    m->par_lo[k] = d->param_lo[k];
    m->par_hi[k] = d->param_hi[k];
    m->par_free[k] = d->param_free ? (d->param_free[k] != 0) : 1;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, d->device) == hipSuccess && cus > 0)
    m->n_cu = cus;
  auto fail = [&](nll_status s) {
    nll_jit_destroy(m);
    return s;
  };
  if (hipModuleLoadData(&m->module, code.data()) != hipSuccess) return fail(NLL_ERR_DEVICE);
  const char* names[4] = {"k_jit_stream_nll", "k_jit_stream_grad", "k_jit_finish_nll", "k_jit_finish_grad"};
  hipFunction_t* slots[4] = {&m->f_stream[0], &m->f_stream[1], &m->f_finish[0], &m->f_finish[1]};
  for (int i = 0; i < 4; ++i)
    if (hipModuleGetFunction(slots[i], m->module, names[i]) != hipSuccess) return fail(NLL_ERR_DEVICE);
  for (int g = 0; g < 2; ++g) {
    int nb = 0;
    if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&nb, m->f_stream[g], kJitThreads, 0) != hipSuccess)
      return fail(NLL_ERR_DEVICE);
    m->stream_blocks_per_cu[g] = std::max(1, std::min(nb, kJitBlocksPerCu));
  }
  const size_t nv = (size_t)d->n_param + 2;
  if ((st = jit_alloc(&m->partials, (size_t)m->n_cu * kJitBlocksPerCu * nv * 2)) != NLL_OK) return fail(st);
  if ((st = jit_alloc(&m->status, 1)) != NLL_OK || (st = jit_alloc(&m->dbad, 1)) != NLL_OK) return fail(st);
  if ((st = jit_alloc(&m->glx, kJitThreads)) != NLL_OK || (st = jit_alloc(&m->glw, kJitThreads)) != NLL_OK)
    return fail(st);
  double hx[kJitThreads], hw[kJitThreads];
  gauss_legendre(kJitThreads, hx, hw);
  if (hipMemcpy(m->glx, hx, sizeof(hx), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->glw, hw, sizeof(hw), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(m->status, 0, sizeof(int)) != hipSuccess)
    return fail(NLL_ERR_DEVICE);
  *out = m;
  return NLL_OK;
}

void nll_jit_destroy(nll_jit_model* m) {
  if (!m) return;
  DeviceGuard guard(m->device);
  (void)hipStreamSynchronize(m->stream);
  if (m->module) (void)hipModuleUnload(m->module);
  jit_free(m->partials);
  jit_free(m->status);
  jit_free(m->dbad);
  jit_free(m->glx);
  jit_free(m->glw);
  delete m;
}

nll_status nll_jit_set_data(nll_jit_model* m, const double* x, int64_t n) {
  if (!m || n < 0 || (n > 0 && (!x || (reinterpret_cast<uintptr_t>(x) & 7u)))) return NLL_ERR_ARG;
  DeviceGuard guard(m->device);
  if (n > 0) {
    unsigned long long bad = 0;
    if (hipMemsetAsync(m->dbad, 0, sizeof(unsigned long long), m->stream) != hipSuccess ||
        launch_check_range(x, n, m->lo, m->hi, m->dbad, m->stream) != hipSuccess ||
        hipMemcpyAsync(&bad, m->dbad, sizeof(bad), hipMemcpyDeviceToHost, m->stream) != hipSuccess ||
        hipStreamSynchronize(m->stream) != hipSuccess)
      return NLL_ERR_DEVICE;
    if (bad) return NLL_ERR_DOMAIN;
  }
  m->x = n > 0 ? x : nullptr;
  m->n = n;
  return NLL_OK;
}

nll_status nll_jit_eval(nll_jit_model* m, const double* theta, double* nll_out, double* grad_out) {
  if (!m || !theta || !nll_out) return NLL_ERR_ARG;
  if (m->n < 0) return NLL_ERR_STATE;
  DeviceGuard guard(m->device);
  JitArgsHost a{};
  a.x = m->x;
  a.n = m->n;
  a.theta = theta;
  a.nll_out = nll_out;
  a.grad_out = grad_out;
  a.partials = m->partials;
  a.status = m->status;
  a.glx = m->glx;
  a.glw = m->glw;
  a.lo = m->lo;
  a.hi = m->hi;
  for (int k = 0; k < kJitMaxParams; ++k) {
    a.par_lo[k] = m->par_lo[k];
    a.par_hi[k] = m->par_hi[k];
    a.par_free[k] = m->par_free[k];
  }
  const int64_t want = (m->n + kJitThreads - 1) / kJitThreads;
  const int g = grad_out ? 1 : 0;
  const int64_t cap = (int64_t)m->n_cu * m->stream_blocks_per_cu[g];
  const int grid = (int)std::max<int64_t>(1, std::min(want, cap));
  a.n_blocks = grid;
  void* args[] = {&a};
  if (hipModuleLaunchKernel(m->f_stream[g], grid, 1, 1, kJitThreads, 1, 1, 0, m->stream, args, nullptr) !=
          hipSuccess ||
      hipModuleLaunchKernel(m->f_finish[g], 1, 1, 1, kJitThreads, 1, 1, 0, m->stream, args, nullptr) != hipSuccess)
    return NLL_ERR_DEVICE;
  return NLL_OK;
}

nll_status nll_jit_sync(nll_jit_model* m, int32_t* status_out) {
  if (!m) return NLL_ERR_ARG;
  DeviceGuard guard(m->device);
  if (hipStreamSynchronize(m->stream) != hipSuccess) return NLL_ERR_DEVICE;
  int bits = 0;
  if (hipMemcpy(&bits, m->status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return NLL_ERR_DEVICE;
  const int zero = 0;
  if (hipMemcpy(m->status, &zero, sizeof(int), hipMemcpyHostToDevice) != hipSuccess) return NLL_ERR_DEVICE;
  nll_status st = NLL_OK;
  if (bits & kStatusParam) st = NLL_ERR_PARAM_RANGE;
  else if (bits & kStatusPdf) st = NLL_ERR_INVALID_PDF;
  if (status_out) *status_out = st;
  return NLL_OK;
}

}  // extern "C"
