// rtc.cpp -- model shapes outside the ahead-of-time registry.  The kernel
// templates of kernels_dev.h are instantiated for the lowered shape and
// compiled for the model's device with hipRTC, the GPU counterpart of the
// just-in-time compilation of Sec. 4 (the sources travel inside the library,
// embedded by the build); the code object is loaded as a module and its
// kernels are launched through the module API with the same argument blocks
// as the ahead-of-time kernels.  A shape compiles once per process and
// device (about 5-15 s); code objects are cached on disk under
// $NLLMI_RTC_CACHE (default $XDG_CACHE_HOME/nllmi or ~/.cache/nllmi; "off"
// disables the cache), keyed by a hash of the sources, the shape and the
// device's architecture.
#include <hip/hip_runtime_api.h>
#include <hip/hiprtc.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "jit_source.h"
#include "rtc.h"
#include "runtime.h"

// the HIP runtime's module launch with start/stop events (hip_ext.h, whose
// kernel-launch templates need the device compiler)
extern "C" hipError_t hipExtModuleLaunchKernel(hipFunction_t f, uint32_t globalWorkSizeX, uint32_t globalWorkSizeY,
                                               uint32_t globalWorkSizeZ, uint32_t localWorkSizeX,
                                               uint32_t localWorkSizeY, uint32_t localWorkSizeZ,
                                               size_t sharedMemBytes, hipStream_t hStream, void** kernelParams,
                                               void** extra, hipEvent_t startEvent, hipEvent_t stopEvent,
                                               uint32_t flags);

namespace nllmi {

// embedded device sources (written by the build from csrc/)
extern const int kRtcHeaderCount;
extern const char* const kRtcHeaderNames[];
extern const char* const kRtcHeaderTexts[];

namespace {

// kernels of one compiled shape
enum KernelId {
  kSingle,       // [grad][u]: 4 entries
  kFinish = 4,   // k_single_finish<M, GRAD, FIT>: (0,0), (1,0), (1,1)
  kFit = 7,      // [u]: 2
  kConsts = 9,
  kFitInit,
  kSets,         // [grad][u]: 4
  kSetsFinish = 15,  // (1,1), (1,0), (0,0)
  kBh = 18,      // [fit][u]: 4
  kBhFinish = 22,    // [fit]: 2
  kW = 24,       // weighted: [grad][u]: 4
  kWFinish = 28,     // (0,0), (1,0), (1,1)
  kWFit = 31,    // [u]: 2
  kNumKernels = 33
};

constexpr int kUs[2] = {2, 4};
constexpr int kRtcMaxAcc = 48;

struct RtcModule {
  std::string name;
  hipModule_t module = nullptr;
  hipFunction_t f[kNumKernels] = {};
  VariantOps ops{};
};

const RtcModule& R(const VariantOps& self) { return *static_cast<const RtcModule*>(self.rtc); }
int u_index(int unroll) { return unroll >= 4 ? 1 : 0; }

size_t pad(hipFunction_t f, int lds_cap) {
  if (lds_cap <= 0) return 0;
  int static_bytes = 0;
  if (hipFuncGetAttribute(&static_bytes, HIP_FUNC_ATTRIBUTE_SHARED_SIZE_BYTES, f) != hipSuccess) return 0;
  return lds_cap > static_bytes ? (size_t)(lds_cap - static_bytes) : 0;
}

// grid blocks of `block` threads; with both events set the launch carries
// them (as hipExtLaunchKernelGGL does for the ahead-of-time kernels)
hipError_t launch(hipFunction_t f, int grid, int block, size_t lds, hipStream_t st, void** args,
                  hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
  if (!f) return hipErrorInvalidDeviceFunction;
  if (ev0 && ev1)
    return hipExtModuleLaunchKernel(f, (uint32_t)grid * (uint32_t)block, 1, 1, (uint32_t)block, 1, 1, lds, st, args,
                                    nullptr, ev0, ev1, 0);
  return hipModuleLaunchKernel(f, (unsigned)grid, 1, 1, (unsigned)block, 1, 1, (unsigned)lds, st, args, nullptr);
}

// --- launchers (the VariantOps interface) -----------------------------------
hipError_t finish_single(hipFunction_t f, const Plan& pl, const SingleArgs& a, int grid, hipStream_t st) {
  int g = grid;
  void* args[] = {const_cast<Plan*>(&pl), const_cast<SingleArgs*>(&a), &g};
  return launch(f, 1, kFinishBlock, 0, st, args);
}

hipError_t op_single(const VariantOps& self, const Plan& pl, const SingleArgs& a, bool grad, int unroll, int grid,
                     int lds_cap, hipStream_t st) {
  const RtcModule& r = R(self);
  hipFunction_t f = r.f[kSingle + 2 * (grad ? 1 : 0) + u_index(unroll)];
  void* args[] = {const_cast<Plan*>(&pl), const_cast<SingleArgs*>(&a)};
  hipError_t e = launch(f, grid, kBlock, pad(f, lds_cap), st, args);
  if (e != hipSuccess) return e;
  return finish_single(r.f[kFinish + (grad ? 1 : 0)], pl, a, grid, st);
}

hipError_t op_single_fit(const VariantOps& self, const Plan& pl, const SingleArgs& a, int unroll, int grid,
                         int lds_cap, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  hipFunction_t f = R(self).f[kFit + u_index(unroll)];
  void* args[] = {const_cast<Plan*>(&pl), const_cast<SingleArgs*>(&a)};
  return launch(f, grid, kBlock, pad(f, lds_cap), st, args, ev0, ev1);
}

hipError_t op_fit_finish(const VariantOps& self, const Plan& pl, const SingleArgs& a, int grid, hipStream_t st) {
  return finish_single(R(self).f[kFinish + 2], pl, a, grid, st);
}

hipError_t op_consts(const VariantOps& self, const Plan& pl, const double* theta, int n_sets, PerTheta* out,
                     double* aux, const double* glx, const double* glw, hipStream_t st) {
  int ns = n_sets;
  void* args[] = {const_cast<Plan*>(&pl), &theta, &ns, &out, &aux, &glx, &glw};
  return launch(R(self).f[kConsts], n_sets, kBlock, 0, st, args);
}

hipError_t op_sets(const VariantOps& self, const Plan& pl, const SetsArgs& a, bool grad, bool fit, int unroll,
                   int grid, int lds_cap, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (a.n_sets <= 0) return hipSuccess;  // the finishing kernel's grid is one block per set
  const RtcModule& r = R(self);
  hipFunction_t f = r.f[kSets + 2 * ((grad || fit) ? 1 : 0) + u_index(unroll)];
  const WorkItem* items = a.items;
  const PerTheta* consts = a.consts;
  const int64_t* chunk_first = a.chunk_first;
  void* sargs[] = {const_cast<Plan*>(&pl), const_cast<SetsArgs*>(&a), &items, &consts, &chunk_first};
  hipError_t e = launch(f, grid, kBlock, pad(f, lds_cap), st, sargs, ev0, ev1);
  void* args[] = {const_cast<Plan*>(&pl), const_cast<SetsArgs*>(&a)};
  if (e != hipSuccess) return e;
  hipFunction_t fin = r.f[kSetsFinish + (fit ? 0 : grad ? 1 : 2)];
  return launch(fin, a.n_sets, self.fin_threads, 0, st, args);
}

hipError_t op_fit_init(const VariantOps& self, const Plan& pl, const double* theta, int n_sets, double eta,
                       const GDState& gd, PerTheta* consts, double* aux, const double* glx, const double* glw,
                       hipStream_t st) {
  int ns = n_sets;
  double et = eta;
  GDState g = gd;
  void* args[] = {const_cast<Plan*>(&pl), &theta, &ns, &et, &g, &consts, &aux, &glx, &glw};
  return launch(R(self).f[kFitInit], n_sets, kBlock, 0, st, args);
}

hipError_t bh(const VariantOps& self, bool fit, const Plan& pl, const SingleArgs& a, int unroll, int grid,
              int lds_cap, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  const RtcModule& r = R(self);
  hipFunction_t f = r.f[kBh + 2 * (fit ? 1 : 0) + u_index(unroll)];
  void* args[] = {const_cast<Plan*>(&pl), const_cast<SingleArgs*>(&a)};
  hipError_t e = launch(f, grid, kBlock, pad(f, lds_cap), st, args, ev0, ev1);
  if (e != hipSuccess) return e;
  return finish_single(r.f[kBhFinish + (fit ? 1 : 0)], pl, a, grid, st);
}

hipError_t op_single_bhhh(const VariantOps& self, const Plan& pl, const SingleArgs& a, int unroll, int grid,
                          int lds_cap, hipStream_t st) {
  return bh(self, false, pl, a, unroll, grid, lds_cap, st, nullptr, nullptr);
}

hipError_t op_single_bhhh_fit(const VariantOps& self, const Plan& pl, const SingleArgs& a, int unroll, int grid,
                              int lds_cap, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  return bh(self, true, pl, a, unroll, grid, lds_cap, st, ev0, ev1);
}

hipError_t op_single_w(const VariantOps& self, const Plan& pl, const SingleArgs& a, bool grad, int unroll, int grid,
                       int lds_cap, hipStream_t st) {
  const RtcModule& r = R(self);
  hipFunction_t f = r.f[kW + 2 * (grad ? 1 : 0) + u_index(unroll)];
  void* args[] = {const_cast<Plan*>(&pl), const_cast<SingleArgs*>(&a)};
  hipError_t e = launch(f, grid, kBlock, pad(f, lds_cap), st, args);
  if (e != hipSuccess) return e;
  return finish_single(r.f[kWFinish + (grad ? 1 : 0)], pl, a, grid, st);
}

hipError_t op_single_w_fit(const VariantOps& self, const Plan& pl, const SingleArgs& a, int unroll, int grid,
                           int lds_cap, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  hipFunction_t f = R(self).f[kWFit + u_index(unroll)];
  void* args[] = {const_cast<Plan*>(&pl), const_cast<SingleArgs*>(&a)};
  return launch(f, grid, kBlock, pad(f, lds_cap), st, args, ev0, ev1);
}

hipError_t op_w_fit_finish(const VariantOps& self, const Plan& pl, const SingleArgs& a, int grid, hipStream_t st) {
  return finish_single(R(self).f[kWFinish + 2], pl, a, grid, st);
}

// --- source, names, compilation ---------------------------------------------
uint64_t fnv1a(uint64_t h, const void* p, size_t n);

// the generated type that holds a formula leaf's expression
std::string jit_functor_name(const std::string& density, int np) {
  uint64_t h = fnv1a(1469598103934665603ull, density.c_str(), density.size() + 1);
  h = fnv1a(h, &np, sizeof(np));
  char hex[17];
  std::snprintf(hex, sizeof(hex), "%016llx", (unsigned long long)h);
  return std::string("nllmi_jit_") + hex;
}

std::string leaf_type(int kind, int np, const std::string& density) {
  switch (kind) {
    case kGauss: return "nllmi::GaussLeaf";
    case kExp: return "nllmi::ExpLeaf";
    case kCheb: return "nllmi::ChebLeaf<" + std::to_string(np) + ">";
    case kCB: return "nllmi::CBLeaf";
    case kArgus: return "nllmi::ArgusLeaf";
    case kJohnson: return "nllmi::JohnsonLeaf";
    case kChi2: return "nllmi::Chi2Leaf";
    case kHypatia: return "nllmi::HypatiaLeaf";
    case kJit: return "nllmi::JitLeaf<" + std::to_string(np) + ",::" + jit_functor_name(density, np) + ">";
    default: return "";
  }
}

const char* tf(bool b) { return b ? "true" : "false"; }

struct Names {
  std::string expr[kNumKernels];
  bool want[kNumKernels] = {};
};

Names kernel_names(const std::string& M, bool bh, bool weighted) {
  Names n;
  auto set = [&](int id, const std::string& s) {
    n.expr[id] = s;
    n.want[id] = true;
  };
  for (int g = 0; g < 2; ++g)
    for (int u = 0; u < 2; ++u) {
      set(kSingle + 2 * g + u,
          "nllmi::k_single<" + M + "," + tf(g) + "," + std::to_string(kUs[u]) + ",false,false>");
      set(kSets + 2 * g + u, "nllmi::k_sets<" + M + "," + tf(g) + "," + std::to_string(kUs[u]) + ">");
    }
  set(kFinish + 0, "nllmi::k_single_finish<" + M + ",false,false,false>");
  set(kFinish + 1, "nllmi::k_single_finish<" + M + ",true,false,false>");
  set(kFinish + 2, "nllmi::k_single_finish<" + M + ",true,true,false>");
  for (int u = 0; u < 2; ++u) set(kFit + u, "nllmi::k_single_fit<" + M + "," + std::to_string(kUs[u]) + ">");
  set(kConsts, "nllmi::k_consts<" + M + ">");
  set(kFitInit, "nllmi::k_fit_init<" + M + ">");
  set(kSetsFinish + 0, "nllmi::k_sets_finish<" + M + ",true,true>");
  set(kSetsFinish + 1, "nllmi::k_sets_finish<" + M + ",true,false>");
  set(kSetsFinish + 2, "nllmi::k_sets_finish<" + M + ",false,false>");
  if (bh) {
    for (int fit = 0; fit < 2; ++fit) {
      for (int u = 0; u < 2; ++u)
        set(kBh + 2 * fit + u,
            "nllmi::k_single<" + M + ",true," + std::to_string(kUs[u]) + "," + tf(fit) + ",true>");
      set(kBhFinish + fit, "nllmi::k_single_finish<" + M + ",true," + tf(fit) + ",true>");
    }
  }
  if (weighted) {
    const std::string W = "nllmi::Weighted<" + M + ">";
    for (int g = 0; g < 2; ++g)
      for (int u = 0; u < 2; ++u)
        set(kW + 2 * g + u, "nllmi::k_single<" + W + "," + tf(g) + "," + std::to_string(kUs[u]) + ",false,false>");
    set(kWFinish + 0, "nllmi::k_single_finish<" + W + ",false,false,false>");
    set(kWFinish + 1, "nllmi::k_single_finish<" + W + ",true,false,false>");
    set(kWFinish + 2, "nllmi::k_single_finish<" + W + ",true,true,false>");
    for (int u = 0; u < 2; ++u) set(kWFit + u, "nllmi::k_single_fit<" + W + "," + std::to_string(kUs[u]) + ">");
  }
  return n;
}

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

std::string cache_dir() {
  const char* e = std::getenv("NLLMI_RTC_CACHE");
  if (e && std::strcmp(e, "off") == 0) return "";
  if (e && *e) return e;
  const char* x = std::getenv("XDG_CACHE_HOME");
  if (x && *x) return std::string(x) + "/nllmi";
  const char* h = std::getenv("HOME");
  if (h && *h) return std::string(h) + "/.cache/nllmi";
  return "";
}

bool make_dirs(const std::string& d) {
  if (d.empty()) return false;
  std::string cur;
  std::stringstream ss(d);
  std::string part;
  if (d[0] == '/') cur = "/";
  while (std::getline(ss, part, '/')) {
    if (part.empty()) continue;
    cur += part + "/";
    if (mkdir(cur.c_str(), 0755) != 0 && errno != EEXIST) return false;
  }
  return true;
}

bool read_file(const std::string& path, std::vector<char>& out) {
  std::ifstream f(path, std::ios::binary);
  if (!f) return false;
  out.assign(std::istreambuf_iterator<char>(f), std::istreambuf_iterator<char>());
  return !out.empty();
}

void write_file_atomic(const std::string& path, const std::vector<char>& data) {
  const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
  {
    std::ofstream f(tmp, std::ios::binary);
    if (!f) return;
    f.write(data.data(), (std::streamsize)data.size());
    if (!f) {
      std::remove(tmp.c_str());
      return;
    }
  }
  if (std::rename(tmp.c_str(), path.c_str()) != 0) std::remove(tmp.c_str());
}

const char* kOptions[] = {"-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};

// The formula leaves' expressions (kJit), after the kernel templates: the
// forward-mode dual numbers, then per formula a type with its value and its
// dual evaluation, as JitLeaf (jit_leaf.h) expects.  Empty without them.
std::string jit_functors(const RtcShape& s) {
  std::string out;
  std::vector<std::string> done;
  for (size_t l = 0; l < s.kind.size(); ++l) {
    if (s.kind[l] != kJit || l >= s.density.size()) continue;
    const std::string name = jit_functor_name(s.density[l], s.np[l]);
    if (std::find(done.begin(), done.end(), name) != done.end()) continue;
    done.push_back(name);
    if (out.empty()) out = jit_dual_source();
    const std::string& e = s.density[l];
    out += "\nstruct " + name + " {\n  template <int N> using D = Dual<N>;\n" +
           "  __device__ static double val(double x, const double* p) { return (double)(" + e + "); }\n" +
           "  template <int N> __device__ static Dual<N> dual(double x, const Dual<N>* p) { return dconst<N>(0.0) + (" +
           e + "); }\n};\n";
  }
  return out;
}

// compile the explicit instantiations of `names` (and their lowered names)
nll_status compile(const std::string& arch, const Names& names, const std::string& extra, std::vector<char>& code,
                   std::vector<std::string>& lowered, std::string& log) {
  std::string src = "#include \"kernels_dev.h\"\n" + extra;
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "nllmi_rtc.hip", kRtcHeaderCount, kRtcHeaderTexts, kRtcHeaderNames) !=
      HIPRTC_SUCCESS)
    return NLL_ERR_DEVICE;
  for (int i = 0; i < kNumKernels; ++i)
    if (names.want[i]) hiprtcAddNameExpression(prog, names.expr[i].c_str());
  std::vector<const char*> opts;
  const std::string a = "--offload-arch=" + arch;
  opts.push_back(a.c_str());
  for (const char* o : kOptions) opts.push_back(o);
  const hiprtcResult r = hiprtcCompileProgram(prog, (int)opts.size(), opts.data());
  size_t ls = 0;
  hiprtcGetProgramLogSize(prog, &ls);
  log.assign(ls, '\0');
  if (ls) hiprtcGetProgramLog(prog, &log[0]);
  if (r != HIPRTC_SUCCESS) {
    hiprtcDestroyProgram(&prog);
    return NLL_ERR_DEVICE;
  }
  lowered.assign(kNumKernels, std::string());
  for (int i = 0; i < kNumKernels; ++i) {
    if (!names.want[i]) continue;
    const char* ln = nullptr;
    if (hiprtcGetLoweredName(prog, names.expr[i].c_str(), &ln) != HIPRTC_SUCCESS || !ln) {
      hiprtcDestroyProgram(&prog);
      return NLL_ERR_DEVICE;
    }
    lowered[i] = ln;
  }
  size_t cs = 0;
  hiprtcGetCodeSize(prog, &cs);
  code.resize(cs);
  hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  return NLL_OK;
}

std::mutex g_mu;
std::map<std::string, std::unique_ptr<RtcModule>> g_modules;  // "device|model type"

}  // namespace

std::string rtc_model_type(const RtcShape& s) {
  std::string m = "nllmi::Model<" + std::to_string(s.K) + "," + std::to_string(s.n_obs);
  for (size_t l = 0; l < s.kind.size(); ++l)
    m += ",nllmi::Slot<" + leaf_type(s.kind[l], s.np[l], l < s.density.size() ? s.density[l] : std::string()) +
         "," + std::to_string(s.obs[l]) + "," + tf(s.root[l] != 0) + ">";
  m += ">";
  if (s.nonflat) m = "nllmi::NonFlat<" + m + ">";
  if (s.precision == 1) m = "nllmi::FP32C<" + m + ">";
  return m;
}

nll_status rtc_compile_check(const RtcShape& s, const std::string& arch, std::string* log) {
  int npt = 0;
  for (size_t l = 0; l < s.kind.size(); ++l) npt += s.np[l];
  const int nvf = (s.K > 1 ? s.K : 0) + npt;
  const Names names = kernel_names(rtc_model_type(s), s.precision == 0 && nvf <= 6,
                                   s.precision == 0 && s.n_obs < kMaxObs);
  std::vector<char> code;
  std::vector<std::string> lowered;
  std::string clog;
  const nll_status st = compile(arch, names, jit_functors(s), code, lowered, clog);
  if (log) *log = clog;
  return st;
}

const VariantOps* rtc_variant(const RtcShape& s, int device, nll_status* status, std::string* log) {
  *status = NLL_OK;
  const int L = (int)s.kind.size();
  if (L < 1 || L > kMaxLeaves || s.K < 1 || s.K > kMaxTerms) {
    *status = NLL_ERR_UNSUPPORTED;
    return nullptr;
  }
  int npt = 0;
  if (s.density.size() != (size_t)L) {
    *status = NLL_ERR_ARG;
    return nullptr;
  }
  for (int l = 0; l < L; ++l) {
    if (leaf_type(s.kind[l], s.np[l], s.density[l]).empty()) {
      *status = NLL_ERR_UNSUPPORTED;
      return nullptr;
    }
    npt += s.np[l];
  }
  const int nt = s.K > 1 ? s.K : 0;
  const int na_grad = 1 + nt + npt + (s.precision == 1 && s.K > 1 ? s.K - 1 : 0);
  // accumulators per record (+ the counters of the FP32 pass) within the
  // kernels' budget, and their LDS transpose (NA + 1 rows of 257 doubles)
  // well inside a block's LDS
  if (na_grad > std::min(kMaxAcc, kRtcMaxAcc)) {
    *status = NLL_ERR_UNSUPPORTED;
    return nullptr;
  }
  const std::string M = rtc_model_type(s);
  const std::string key = std::to_string(device) + "|" + M;
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_modules.find(key);
  if (it != g_modules.end()) return &it->second->ops;

  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    *status = NLL_ERR_DEVICE;
    return nullptr;
  }
  std::string arch = prop.gcnArchName;
  const size_t colon = arch.find(':');  // feature suffixes (":sramecc+:xnack-") stay off
  if (colon != std::string::npos) arch.resize(colon);
  const int nvf = nt + npt;
  const bool bh = s.precision == 0 && nvf <= 6;
  const bool weighted = s.precision == 0 && s.n_obs < kMaxObs;
  const Names names = kernel_names(M, bh, weighted);

  uint64_t h = 1469598103934665603ull;
  for (int i = 0; i < kRtcHeaderCount; ++i) {
    h = fnv1a(h, kRtcHeaderNames[i], std::strlen(kRtcHeaderNames[i]) + 1);
    h = fnv1a(h, kRtcHeaderTexts[i], std::strlen(kRtcHeaderTexts[i]) + 1);
  }
  for (int i = 0; i < kNumKernels; ++i) h = fnv1a(h, names.expr[i].c_str(), names.expr[i].size() + 1);
  const std::string extra = jit_functors(s);
  h = fnv1a(h, extra.c_str(), extra.size() + 1);
  for (const char* o : kOptions) h = fnv1a(h, o, std::strlen(o) + 1);
  h = fnv1a(h, arch.c_str(), arch.size() + 1);
  int rtc_ver[2] = {0, 0};
  hiprtcVersion(&rtc_ver[0], &rtc_ver[1]);
  h = fnv1a(h, rtc_ver, sizeof(rtc_ver));
  char hex[17];
  std::snprintf(hex, sizeof(hex), "%016llx", (unsigned long long)h);
  const std::string dir = cache_dir();
  const std::string path = dir.empty() ? "" : dir + "/" + hex + ".co";
  const std::string lpath = dir.empty() ? "" : dir + "/" + hex + ".names";

  std::vector<char> code;
  std::vector<std::string> lowered;
  bool cached = false;
  if (!path.empty() && read_file(path, code)) {
    std::ifstream f(lpath);
    lowered.assign(kNumKernels, std::string());
    int got = 0;
    for (int i = 0; i < kNumKernels && f; ++i) {
      std::string line;
      if (!std::getline(f, line)) break;
      lowered[i] = line;
      ++got;
    }
    cached = got == kNumKernels;
    for (int i = 0; i < kNumKernels && cached; ++i) cached = names.want[i] == !lowered[i].empty();
  }
  if (!cached) {
    std::string clog;
    const nll_status st = compile(arch, names, extra, code, lowered, clog);
    if (log) *log = clog;
    if (st != NLL_OK) {
      *status = st;
      return nullptr;
    }
    if (!path.empty() && make_dirs(dir)) {
      std::string text;
      for (int i = 0; i < kNumKernels; ++i) text += lowered[i] + "\n";
      write_file_atomic(lpath, std::vector<char>(text.begin(), text.end()));
      write_file_atomic(path, code);
    }
  }

  std::unique_ptr<RtcModule> r(new RtcModule());
  r->name = "rtc:" + M;
  for (const char* p : {"nllmi::"}) {
    size_t pos;
    while ((pos = r->name.find(p)) != std::string::npos) r->name.erase(pos, std::strlen(p));
  }
  if (hipModuleLoadData(&r->module, code.data()) != hipSuccess) {
    *status = NLL_ERR_DEVICE;
    return nullptr;
  }
  for (int i = 0; i < kNumKernels; ++i) {
    if (!names.want[i]) continue;
    if (hipModuleGetFunction(&r->f[i], r->module, lowered[i].c_str()) != hipSuccess) {
      (void)hipModuleUnload(r->module);
      *status = NLL_ERR_DEVICE;
      return nullptr;
    }
  }
  VariantOps& v = r->ops;
  v.name = r->name.c_str();
  v.n_leaf = L;
  v.K = s.K;
  v.nobs = s.n_obs;
  v.na_grad = na_grad;
  for (int l = 0; l < L; ++l) {
    v.kind[l] = s.kind[l];
    v.obs[l] = s.obs[l];
    v.root[l] = s.root[l];
    v.np[l] = s.np[l];
  }
  v.precision = s.precision;
  int n_nonroot = 0;
  for (int l = 0; l < L; ++l) n_nonroot += s.root[l] ? 0 : 1;
  v.flat = (s.K > 1 && n_nonroot == s.K && !s.nonflat) ? 1 : 0;
  v.rtc = r.get();
  v.aux = 0;
  for (int l = 0; l < L; ++l)
    if (s.kind[l] == kHypatia) v.aux = 1;
  v.fin_threads = (v.aux || L > 4) ? kBlock : kBlock / 2;  // as finish_threads<M> (kernels_dev.h)
  v.single = &op_single;
  v.single_fit = &op_single_fit;
  v.fit_finish = &op_fit_finish;
  v.consts = &op_consts;
  v.sets = &op_sets;
  v.fit_init = &op_fit_init;
  if (bh) {
    v.single_bhhh = &op_single_bhhh;
    v.single_bhhh_fit = &op_single_bhhh_fit;
    v.bhhh_record = na_grad + 1 + nvf * (nvf + 1) / 2;
  }
  if (weighted) {
    v.single_w = &op_single_w;
    v.single_w_fit = &op_single_w_fit;
    v.w_fit_finish = &op_w_fit_finish;
  }
  const VariantOps* out = &r->ops;
  g_modules[key] = std::move(r);
  return out;
}

}  // namespace nllmi
