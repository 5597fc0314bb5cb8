// host_hf.cpp -- the C ABI of the binned template likelihood: validation
// of the model descriptor, the library's delta templates, launches and
// status reporting.
#include <hip/hip_runtime_api.h>

#include <cfloat>
#include <cmath>
#include <new>

#include "histfactory.h"
#include "kernels.h"
#include "nll.h"
#include "runtime.h"

using namespace nllmi;

struct nll_hf_model {
  int device = 0;
  hipStream_t stream = nullptr;
  int n_cu = 256;
  HFPlan plan{};
  int histo_caller[kHfMaxHisto] = {};  // sorted histosys -> caller's template index
  int64_t n_bins = 0;
  const double* counts = nullptr;
  const double* nominal[kHfMaxSamples] = {};
  double* deltas = nullptr;      // per histosys: up - T, then T - down (n_bins each)
  double* partials = nullptr;    // grid * kHfNV double-double pairs
  int* status = nullptr;
  unsigned long long* dbad = nullptr;
  bool have_data = false;
  double* stat_tau = nullptr;    // per-bin statistical parameters: 1/sigma_b^2, -1 where none
  bool have_stat = false;
};

namespace {

template <class T>
nll_status hf_alloc(T** p, size_t count) {
  *p = nullptr;
  const hipError_t e = hipMalloc(reinterpret_cast<void**>(p), (count ? count : 1) * sizeof(T));
  if (e == hipSuccess) return NLL_OK;
  return e == hipErrorOutOfMemory ? NLL_ERR_OOM : NLL_ERR_DEVICE;
}

template <class T>
void hf_free(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// persistent grid: at most kHfBlocksPerCu blocks per CU (the partials
// buffer holds exactly that many records).  Measured at 2e6 and 2e7 bins:
// one block per CU streams ~20 % slower; three stream no faster and the
// finisher pays a third round trip for the records.
constexpr int kHfBlocksPerCu = 2;

int hf_grid(const nll_hf_model* m) {
  const int64_t want = (m->n_bins + kBlock - 1) / kBlock;
  const int64_t cap = (int64_t)m->n_cu * kHfBlocksPerCu;
  return (int)(want < 1 ? 1 : want > cap ? cap : want);
}

bool aligned(const void* p) { return p && (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

}  // namespace

extern "C" {

nll_status nll_hf_create(const nll_hf_desc* d, nll_hf_model** out) {
  if (!d || !out) return NLL_ERR_ARG;
  *out = nullptr;
  if (d->n_bins < 0 || d->n_samples < 1 || d->n_param < 1 || d->n_modifiers < 0) return NLL_ERR_ARG;
  if (!d->param_lo || !d->param_hi || (d->n_modifiers > 0 && !d->modifiers)) return NLL_ERR_ARG;
  if (d->n_samples > kHfMaxSamples || d->n_param > kMaxParams) return NLL_ERR_UNSUPPORTED;
  HFPlan pl{};
  pl.n_samples = d->n_samples;
  pl.n_param = d->n_param;
  for (int p = 0; p < d->n_param; ++p) {
    if (!(d->param_lo[p] <= d->param_hi[p])) return NLL_ERR_ARG;
    pl.par_lo[p] = d->param_lo[p];
    pl.par_hi[p] = d->param_hi[p];
    pl.par_free[p] = d->param_free ? (d->param_free[p] != 0) : 1;
    pl.par_constrained[p] = d->param_constrained ? (d->param_constrained[p] != 0) : 0;
    const double mean = d->param_mean ? d->param_mean[p] : 0.0;
    const double sig = d->param_sigma ? d->param_sigma[p] : 1.0;
    if (pl.par_constrained[p] && !(std::isfinite(mean) && sig > 0.0 && std::isfinite(sig))) return NLL_ERR_ARG;
    pl.par_mean[p] = mean;
    pl.par_ivar[p] = 1.0 / (sig * sig);
  }
  int n_nf = 0, n_ns = 0, n_hs = 0, n_smooth_hs = 0;
  for (int i = 0; i < d->n_modifiers; ++i) {
    const nll_hf_modifier& md = d->modifiers[i];
    if (md.sample < 0 || md.sample >= d->n_samples || md.param < 0 || md.param >= d->n_param) return NLL_ERR_ARG;
    if (md.interp != 0 && md.interp != 1) return NLL_ERR_ARG;
    if (md.type == NLL_HF_HISTOSYS && md.interp == 1) ++n_smooth_hs;
    if (md.type == NLL_HF_NORMFACTOR) {
      ++n_nf;
    } else if (md.type == NLL_HF_NORMSYS) {
      if (!(md.hi > 0.0 && md.lo > 0.0 && std::isfinite(md.hi) && std::isfinite(md.lo))) return NLL_ERR_ARG;
      ++n_ns;
    } else if (md.type == NLL_HF_HISTOSYS) {
      ++n_hs;
    } else {
      return NLL_ERR_ARG;
    }
  }
  if (n_nf > kHfMaxNormfactor || n_ns > kHfMaxNormsys || n_hs > kHfMaxHisto) return NLL_ERR_UNSUPPORTED;
  // a smooth histosys: both delta templates of every histosys are summed
  // apart, two record slots each
  if (n_smooth_hs > 0 && n_hs > kHfPolyHisto) return NLL_ERR_UNSUPPORTED;
  pl.smooth_histo = n_smooth_hs > 0 ? 1 : 0;
  // each kind sorted by sample (stable), with per-sample ranges; histo_caller
  // maps a sorted histosys to its position in the caller's template order
  int histo_caller[kHfMaxHisto] = {};
  for (int s = 0; s < d->n_samples; ++s) {
    pl.nf_start[s] = pl.n_normfactor;
    pl.ns_start[s] = pl.n_normsys;
    pl.hs_start[s] = pl.n_histo;
    int caller_h = 0;
    for (int i = 0; i < d->n_modifiers; ++i) {
      const nll_hf_modifier& md = d->modifiers[i];
      if (md.type == NLL_HF_HISTOSYS) ++caller_h;
      if (md.sample != s) continue;
      if (md.type == NLL_HF_NORMFACTOR) {
        pl.nf_sample[pl.n_normfactor] = s;
        pl.nf_param[pl.n_normfactor++] = md.param;
      } else if (md.type == NLL_HF_NORMSYS) {
        pl.ns_sample[pl.n_normsys] = s;
        pl.ns_param[pl.n_normsys] = md.param;
        pl.ns_code[pl.n_normsys] = md.interp;
        pl.ns_lnhi[pl.n_normsys] = std::log(md.hi);
        pl.ns_lnlo[pl.n_normsys++] = std::log(md.lo);
      } else {
        histo_caller[pl.n_histo] = caller_h - 1;
        pl.hs_code[pl.n_histo] = md.interp;
        pl.histo_sample[pl.n_histo] = s;
        pl.histo_param[pl.n_histo++] = md.param;
      }
    }
  }
  pl.nf_start[d->n_samples] = pl.n_normfactor;
  pl.ns_start[d->n_samples] = pl.n_normsys;
  pl.hs_start[d->n_samples] = pl.n_histo;
  // per parameter: the contribution slots of the modifiers it drives
  int n_slot = 0;
  for (int p = 0; p < d->n_param; ++p) {
    pl.par_start[p] = n_slot;
    for (int i = 0; i < pl.n_normfactor; ++i)
      if (pl.nf_param[i] == p) pl.par_slot[n_slot++] = i;
    for (int k = 0; k < pl.n_normsys; ++k)
      if (pl.ns_param[k] == p) pl.par_slot[n_slot++] = kHfMaxNormfactor + k;
    for (int h = 0; h < pl.n_histo; ++h)
      if (pl.histo_param[h] == p) pl.par_slot[n_slot++] = kHfMaxNormfactor + kHfMaxNormsys + h;
  }
  pl.par_start[d->n_param] = n_slot;
  DeviceGuard guard(d->device);
  nll_hf_model* m = new (std::nothrow) nll_hf_model();
  if (!m) return NLL_ERR_OOM;
  m->device = d->device;
  m->stream = reinterpret_cast<hipStream_t>(d->stream);
  m->plan = pl;
  for (int h = 0; h < kHfMaxHisto; ++h) m->histo_caller[h] = histo_caller[h];
  m->n_bins = d->n_bins;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, d->device) == hipSuccess && cus > 0)
    m->n_cu = cus;
  nll_status st;
  if ((st = hf_alloc(&m->deltas, 2 * (size_t)pl.n_histo * (size_t)d->n_bins)) != NLL_OK ||
      (st = hf_alloc(&m->partials, (size_t)m->n_cu * kHfBlocksPerCu * kHfNV * 2)) != NLL_OK ||
      (st = hf_alloc(&m->status, 1)) != NLL_OK || (st = hf_alloc(&m->dbad, 1)) != NLL_OK) {
    nll_hf_destroy(m);
    return st;
  }
  if (hipMemset(m->status, 0, sizeof(int)) != hipSuccess) {
    nll_hf_destroy(m);
    return NLL_ERR_DEVICE;
  }
  *out = m;
  return NLL_OK;
}

void nll_hf_destroy(nll_hf_model* m) {
  if (!m) return;
  DeviceGuard guard(m->device);
  (void)hipStreamSynchronize(m->stream);
  hf_free(m->deltas);
  hf_free(m->partials);
  hf_free(m->status);
  hf_free(m->dbad);
  hf_free(m->stat_tau);
  delete m;
}

nll_status nll_hf_set_data(nll_hf_model* m, const double* counts, const double* const* nominal,
                           const double* const* up, const double* const* down) {
  if (!m) return NLL_ERR_ARG;
  const int S = m->plan.n_samples, H = m->plan.n_histo;
  const int64_t B = m->n_bins;
  if (B > 0) {
    if (!aligned(counts) || !nominal) return NLL_ERR_ARG;
    for (int s = 0; s < S; ++s)
      if (!aligned(nominal[s])) return NLL_ERR_ARG;
    if (H > 0 && (!up || !down)) return NLL_ERR_ARG;
    for (int h = 0; h < H; ++h)
      if (!aligned(up[h]) || !aligned(down[h])) return NLL_ERR_ARG;
  }
  DeviceGuard guard(m->device);
  m->have_data = false;
  if (B > 0) {
    if (hipMemsetAsync(m->dbad, 0, sizeof(unsigned long long), m->stream) != hipSuccess) return NLL_ERR_DEVICE;
    if (launch_check_range(counts, B, 0.0, DBL_MAX, m->dbad, m->stream) != hipSuccess) return NLL_ERR_DEVICE;
    for (int h = 0; h < H; ++h) {
      double* dup = m->deltas + (size_t)(2 * h) * (size_t)B;
      double* ddn = m->deltas + (size_t)(2 * h + 1) * (size_t)B;
      const int j = m->histo_caller[h];
      if (launch_hf_deltas(nominal[m->plan.histo_sample[h]], up[j], down[j], B, dup, ddn, m->stream) != hipSuccess)
        return NLL_ERR_DEVICE;
    }
    unsigned long long bad = 0;
    if (hipMemcpyAsync(&bad, m->dbad, sizeof(bad), hipMemcpyDeviceToHost, m->stream) != hipSuccess ||
        hipStreamSynchronize(m->stream) != hipSuccess)
      return NLL_ERR_DEVICE;
    if (bad) return NLL_ERR_DOMAIN;
  }
  m->counts = B > 0 ? counts : nullptr;
  for (int s = 0; s < kHfMaxSamples; ++s) m->nominal[s] = (B > 0 && s < S) ? nominal[s] : nullptr;
  m->have_data = true;
  return NLL_OK;
}

static nll_status hf_set_bin_params(nll_hf_model* m, uint32_t sample_mask, const double* sigma, int kind) {
  if (!m) return NLL_ERR_ARG;
  const int S = m->plan.n_samples;
  if (sample_mask == 0 || (S < 32 && (sample_mask >> S) != 0)) return NLL_ERR_ARG;
  if (m->n_bins > 0 && !aligned(sigma)) return NLL_ERR_ARG;
  DeviceGuard guard(m->device);
  if (!m->stat_tau) {
    const nll_status st = hf_alloc(&m->stat_tau, (size_t)m->n_bins);
    if (st != NLL_OK) return st;
  }
  if (m->n_bins > 0 && launch_hf_tau(sigma, m->n_bins, m->stat_tau, m->stream) != hipSuccess) return NLL_ERR_DEVICE;
  m->plan.stat_mask = (int32_t)sample_mask;
  m->plan.stat_kind = kind;
  m->have_stat = true;
  return NLL_OK;
}

nll_status nll_hf_set_staterror(nll_hf_model* m, uint32_t sample_mask, const double* sigma) {
  return hf_set_bin_params(m, sample_mask, sigma, 0);
}

nll_status nll_hf_set_shapesys(nll_hf_model* m, uint32_t sample_mask, const double* sigma) {
  return hf_set_bin_params(m, sample_mask, sigma, 1);
}

static nll_status hf_eval_impl(nll_hf_model* m, const double* theta, const double* gamma, double* nll_out,
                               double* grad_out, double* grad_gamma) {
  DeviceGuard guard(m->device);
  HFArgs a{};
  a.n_bins = m->n_bins;
  a.counts = m->counts;
  for (int s = 0; s < kHfMaxSamples; ++s) a.nominal[s] = m->nominal[s];
  for (int h = 0; h < m->plan.n_histo; ++h) {
    a.dup[h] = m->deltas + (size_t)(2 * h) * (size_t)m->n_bins;
    a.ddn[h] = m->deltas + (size_t)(2 * h + 1) * (size_t)m->n_bins;
  }
  a.theta = theta;
  a.nll_out = nll_out;
  a.grad_out = grad_out;
  a.partials = m->partials;
  a.status = m->status;
  a.gamma = gamma;
  a.stat_tau = gamma ? m->stat_tau : nullptr;
  a.grad_gamma = gamma ? grad_gamma : nullptr;
  const bool grad = grad_out != nullptr || a.grad_gamma != nullptr;
  const hipError_t e = launch_hf_eval(m->plan, a, grad, hf_grid(m), m->stream);
  return e == hipSuccess ? NLL_OK : NLL_ERR_DEVICE;
}

nll_status nll_hf_eval(nll_hf_model* m, const double* theta, double* nll_out, double* grad_out) {
  if (!m || !theta || !nll_out) return NLL_ERR_ARG;
  if (!m->have_data) return NLL_ERR_STATE;
  return hf_eval_impl(m, theta, nullptr, nll_out, grad_out, nullptr);
}

nll_status nll_hf_eval_stat(nll_hf_model* m, const double* theta, const double* gamma, double* nll_out,
                            double* grad_out, double* grad_gamma) {
  if (!m || !theta || !nll_out) return NLL_ERR_ARG;
  if (m->n_bins > 0 && (!aligned(gamma) || (grad_gamma && !aligned(grad_gamma)))) return NLL_ERR_ARG;
  if (!m->have_data || !m->have_stat) return NLL_ERR_STATE;
  if (m->n_bins == 0) return hf_eval_impl(m, theta, nullptr, nll_out, grad_out, nullptr);
  return hf_eval_impl(m, theta, gamma, nll_out, grad_out, grad_gamma);
}

nll_status nll_hf_sync(nll_hf_model* m, int32_t* status_out) {
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
