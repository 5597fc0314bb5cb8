// host.cpp -- the C ABI of libnllmi: model validation, lowering of the
// graph onto a compiled kernel shape, device scratch, launches, the
// recorded HIP graph of a batched fit, status reporting.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "kernels.h"
#include "nll.h"
#include "plan.h"
#include "rtc.h"
#include "runtime.h"

using namespace nllmi;

// ---------------------------------------------------------------------------
// registry of compiled shapes, per-device Gauss-Legendre tables
// ---------------------------------------------------------------------------
static const std::vector<VariantOps>& registry() {
  static std::vector<VariantOps> reg;
  static std::once_flag once;
  std::call_once(once, [] {
    register_variants_single(reg);
    register_variants_mixture(reg);
    register_variants_2d(reg);
    register_variants_fp32c_1d(reg);
    register_variants_fp32c_2d(reg);
    register_variants_johnson(reg);
    register_variants_chi2(reg);
    register_variants_hypatia(reg);
  });
  return reg;
}

static nll_status gl_table(int device, GLTable* out) {
  static std::mutex mu;
  static std::map<int, GLTable> tables;
  std::lock_guard<std::mutex> lock(mu);
  auto it = tables.find(device);
  if (it != tables.end()) {
    *out = it->second;
    return NLL_OK;
  }
  double hx[256], hw[256];
  gauss_legendre(256, hx, hw);
  GLTable t;
  if (hipMalloc(&t.x, sizeof(hx)) != hipSuccess || hipMalloc(&t.w, sizeof(hw)) != hipSuccess)
    return NLL_ERR_OOM;
  if (hipMemcpy(t.x, hx, sizeof(hx), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t.w, hw, sizeof(hw), hipMemcpyHostToDevice) != hipSuccess)
    return NLL_ERR_DEVICE;
  tables[device] = t;
  *out = t;
  return NLL_OK;
}

// ---------------------------------------------------------------------------
// the model object
// ---------------------------------------------------------------------------
namespace {

nll_status dev_err(hipError_t e) {
  if (e == hipSuccess) return NLL_OK;
  return e == hipErrorOutOfMemory ? NLL_ERR_OOM : NLL_ERR_DEVICE;
}

template <class T>
nll_status dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return dev_err(hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T)));
}

template <class T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

int expected_params(int kind, int np) {
  switch (kind) {
    case NLL_GAUSS: return 2;
    case NLL_EXP: return 1;
    case NLL_CHEB: return (np >= 1 && np <= 8) ? np : -1;
    case NLL_CB: return 4;
    case NLL_ARGUS: return 2;
    case NLL_JOHNSON: return 4;
    case NLL_CHI2: return 1;
    case NLL_HYPATIA: return 9;
    case NLL_JIT: return (np >= 1 && np <= kJitMaxLeafParams) ? np : -1;
    default: return -1;
  }
}

bool is_leaf(int kind) {
  return (kind >= NLL_GAUSS && kind <= NLL_ARGUS) || kind == NLL_JOHNSON || kind == NLL_CHI2 || kind == NLL_HYPATIA ||
         kind == NLL_JIT;
}

// A formula leaf's expression: present, at most 4096 characters, and every
// parameter reference p[k] a literal index below the leaf's parameter count
// (the expression is compiled as given; an index past the leaf's
// parameters would read past them).
nll_status check_density(const char* e, int np) {
  if (!e) return NLL_ERR_ARG;
  const size_t n = std::strlen(e);
  if (n == 0) return NLL_ERR_ARG;
  if (n > 4096) return NLL_ERR_UNSUPPORTED;
  auto ident = [](char c) { return std::isalnum((unsigned char)c) || c == '_'; };
  for (size_t i = 0; i + 1 < n; ++i) {
    if (e[i] != 'p' || (i > 0 && ident(e[i - 1]))) continue;
    size_t j = i + 1;
    while (j < n && e[j] == ' ') ++j;
    if (j >= n || e[j] != '[') continue;
    ++j;
    while (j < n && e[j] == ' ') ++j;
    if (j >= n || !std::isdigit((unsigned char)e[j])) return NLL_ERR_ARG;
    long k = 0;
    while (j < n && std::isdigit((unsigned char)e[j]) && k < 1000) k = 10 * k + (e[j++] - '0');
    while (j < n && e[j] == ' ') ++j;
    if (j >= n || e[j] != ']' || k >= np) return NLL_ERR_ARG;
  }
  return NLL_OK;
}

// ---------------------------------------------------------------------------
// lowering: graph -> sum of products of leaves
// ---------------------------------------------------------------------------
struct Term {
  uint32_t mask = 0;                       // leaves (by position in `leaves`)
  std::vector<std::pair<int, int>> refs;   // (sum position, child index)
};

struct Lowering {
  const nll_model_desc* d = nullptr;
  std::vector<int> leaves, sums;   // node indices, in node order
  std::vector<int> leaf_pos, sum_pos;
  std::vector<unsigned> obs_mask;  // per node

  nll_status validate() {
    const nll_model_desc& D = *d;
    if (D.n_obs < 1 || D.n_obs > NLL_MAX_OBS || !D.obs_lo || !D.obs_hi) return NLL_ERR_ARG;
    if (D.n_param < 1 || D.n_param > NLL_MAX_PARAMS || !D.param_lo || !D.param_hi) return NLL_ERR_ARG;
    if (D.n_node < 1 || D.n_node > NLL_MAX_NODES || !D.nodes) return NLL_ERR_ARG;
    if (D.root < 0 || D.root >= D.n_node) return NLL_ERR_ARG;
    if (D.precision != NLL_FP64 && D.precision != NLL_FP32C) return NLL_ERR_ARG;
    for (int o = 0; o < D.n_obs; ++o)
      if (!(std::isfinite(D.obs_lo[o]) && std::isfinite(D.obs_hi[o]) && D.obs_lo[o] < D.obs_hi[o])) return NLL_ERR_ARG;
    for (int k = 0; k < D.n_param; ++k)
      if (!(D.param_lo[k] <= D.param_hi[k])) return NLL_ERR_ARG;
    if (D.extended && D.yield_param >= D.n_param) return NLL_ERR_ARG;  // < 0: the root's sum of yields
    obs_mask.assign(D.n_node, 0u);
    int n_hypatia = 0;
    for (int i = 0; i < D.n_node; ++i) {
      const nll_node_desc& nd = D.nodes[i];
      if (nd.n_param < 0 || nd.n_param > NLL_NODE_MAX_PARAMS) return NLL_ERR_ARG;
      if (nd.n_child < 0 || nd.n_child > NLL_NODE_MAX_CHILDREN) return NLL_ERR_ARG;
      for (int k = 0; k < nd.n_param; ++k)
        if (nd.param[k] < 0 || nd.param[k] >= D.n_param) return NLL_ERR_ARG;
      if (is_leaf(nd.kind)) {
        if (nd.obs < 0 || nd.obs >= D.n_obs || nd.n_child != 0) return NLL_ERR_ARG;
        if (expected_params(nd.kind, nd.n_param) != nd.n_param) return NLL_ERR_ARG;
        if (nd.norm < NLL_NORM_ANALYTIC || nd.norm > NLL_NORM_GL256_SINGLE) return NLL_ERR_ARG;
        if (nd.kind == NLL_ARGUS && D.obs_lo[nd.obs] < 0.0) return NLL_ERR_UNSUPPORTED;
        if (nd.kind == NLL_CHI2 && (D.obs_lo[nd.obs] < 0.0 || D.obs_hi[nd.obs] > 1000.0)) return NLL_ERR_UNSUPPORTED;
        // Hypatia2: its per-point tables sit beside the constants, one set
        // per model, and the FP32-compensated pass has no form of it
        if (nd.kind == NLL_HYPATIA && (++n_hypatia > 1 || D.precision != NLL_FP64)) return NLL_ERR_UNSUPPORTED;
        // a formula leaf: FP64 only (its expression has no FP32 form)
        if (nd.kind == NLL_JIT) {
          const nll_status ds = check_density(nd.density, nd.n_param);
          if (ds != NLL_OK) return ds;
          if (D.precision != NLL_FP64) return NLL_ERR_UNSUPPORTED;
        }
        obs_mask[i] = 1u << nd.obs;
      } else if (nd.kind == NLL_SUM || nd.kind == NLL_PROD) {
        // a sum takes fractions f_1..f_{k-1} or yields nu_1..nu_k
        if (nd.kind == NLL_SUM && (nd.n_child < 2 || (nd.n_param != nd.n_child - 1 && nd.n_param != nd.n_child)))
          return NLL_ERR_ARG;
        if (nd.kind == NLL_PROD && (nd.n_child < 1 || nd.n_param != 0)) return NLL_ERR_ARG;
        unsigned acc = 0;
        for (int j = 0; j < nd.n_child; ++j) {
          const int c = nd.child[j];
          if (c < 0 || c >= i) return NLL_ERR_ARG;  // topological order
          if (nd.kind == NLL_SUM) {
            if (j > 0 && obs_mask[c] != acc) return NLL_ERR_ARG;  // same observables
            acc = obs_mask[c];
          } else {
            if (obs_mask[c] & acc) return NLL_ERR_ARG;  // disjoint observables
            acc |= obs_mask[c];
          }
        }
        obs_mask[i] = acc;
      } else {
        return NLL_ERR_ARG;
      }
    }
    if (obs_mask[D.root] != (1u << D.n_obs) - 1u) return NLL_ERR_ARG;  // every observable used
    return NLL_OK;
  }

  void collect(int i, std::vector<char>& seen) {
    if (seen[i]) return;
    seen[i] = 1;
    const nll_node_desc& nd = d->nodes[i];
    for (int j = 0; j < nd.n_child; ++j) collect(nd.child[j], seen);
  }

  std::vector<Term> expand(int i) {
    const nll_node_desc& nd = d->nodes[i];
    if (is_leaf(nd.kind)) return {Term{1u << leaf_pos[i], {}}};
    std::vector<Term> out;
    if (nd.kind == NLL_SUM) {
      for (int j = 0; j < nd.n_child; ++j)
        for (Term t : expand(nd.child[j])) {
          t.refs.push_back({sum_pos[i], j});
          out.push_back(t);
        }
      return out;
    }
    out.push_back(Term{});
    for (int j = 0; j < nd.n_child; ++j) {
      std::vector<Term> next;
      for (const Term& a : out)
        for (const Term& b : expand(nd.child[j])) {
          Term t = a;
          t.mask |= b.mask;
          t.refs.insert(t.refs.end(), b.refs.begin(), b.refs.end());
          next.push_back(t);
        }
      out.swap(next);
    }
    return out;
  }
};

// Match the lowered leaves against a compiled shape: perm[slot] = leaf.
bool match_variant(const VariantOps& v, const std::vector<int>& kind, const std::vector<int>& obs,
                   const std::vector<int>& root, const std::vector<int>& np, int K, int n_obs, int precision,
                   std::vector<int>& perm) {
  const int L = (int)kind.size();
  if (v.n_leaf != L || v.K != K || v.nobs != n_obs || v.precision != precision) return false;
  std::vector<int> p(L);
  for (int i = 0; i < L; ++i) p[i] = i;
  do {
    bool ok = true;
    for (int s = 0; s < L && ok; ++s) {
      const int l = p[s];
      ok = v.kind[s] == kind[l] && v.obs[s] == obs[l] && v.root[s] == root[l] && v.np[s] == np[l];
    }
    if (ok) {
      perm = p;
      return true;
    }
  } while (std::next_permutation(p.begin(), p.end()));
  return false;
}

nll_status build_plan(const nll_model_desc& D, Plan& pl, const VariantOps** ops_out) {
  Lowering lw;
  lw.d = &D;
  nll_status st = lw.validate();
  if (st != NLL_OK) return st;
  std::vector<char> seen(D.n_node, 0);
  lw.collect(D.root, seen);
  lw.leaf_pos.assign(D.n_node, -1);
  lw.sum_pos.assign(D.n_node, -1);
  for (int i = 0; i < D.n_node; ++i) {
    if (!seen[i]) continue;
    if (is_leaf(D.nodes[i].kind)) {
      lw.leaf_pos[i] = (int)lw.leaves.size();
      lw.leaves.push_back(i);
    } else if (D.nodes[i].kind == NLL_SUM) {
      lw.sum_pos[i] = (int)lw.sums.size();
      lw.sums.push_back(i);
    }
  }
  const int L = (int)lw.leaves.size();
  if (L > kMaxLeaves || (int)lw.sums.size() > kMaxSums) return NLL_ERR_UNSUPPORTED;
  std::vector<Term> terms = lw.expand(D.root);
  const int K = (int)terms.size();
  if (K > kMaxTerms) return NLL_ERR_UNSUPPORTED;
  for (const Term& t : terms)
    if ((int)t.refs.size() > kMaxPathRefs) return NLL_ERR_UNSUPPORTED;

  std::vector<int> kind(L), obs(L), root(L), np(L);
  std::vector<std::string> density(L);
  for (int l = 0; l < L; ++l) {
    const nll_node_desc& nd = D.nodes[lw.leaves[l]];
    kind[l] = nd.kind;
    if (nd.kind == NLL_JIT) density[l] = nd.density;
    obs[l] = nd.obs;
    np[l] = nd.n_param;
    bool all = true;
    for (const Term& t : terms) all = all && ((t.mask >> l) & 1u);
    root[l] = all ? 1 : 0;
  }
  // Flat structure: as many non-root leaves as terms, and each term holds
  // exactly one of them (a sum of leaves, possibly times root factors).
  // The kernels then take term k from the k-th non-root slot; otherwise the
  // term masks decide.
  int n_nonroot = 0;
  for (int l = 0; l < L; ++l) n_nonroot += root[l] ? 0 : 1;
  std::vector<int> term_of_leaf(L, -1);
  bool flat_struct = K > 1 && n_nonroot == K;
  for (int l = 0; l < L && flat_struct; ++l) {
    if (root[l]) continue;
    int count = 0;
    for (int k = 0; k < K; ++k) {
      int nr = 0;
      for (int q = 0; q < L; ++q)
        if (((terms[k].mask >> q) & 1u) && !root[q]) ++nr;
      if (nr == 1 && ((terms[k].mask >> l) & 1u)) {
        term_of_leaf[l] = k;
        ++count;
      }
    }
    flat_struct = count == 1;
  }
  const int need_flat = flat_struct ? 1 : 0;
  std::vector<int> perm;
  const VariantOps* found = nullptr;
  for (const VariantOps& v : registry()) {
    if (v.flat == need_flat && match_variant(v, kind, obs, root, np, K, D.n_obs, D.precision, perm)) {
      found = &v;
      break;
    }
  }
  if (!found) {
    // any other shape: the same kernel templates compiled for it at run time
    RtcShape shape;
    shape.kind = kind;
    shape.obs = obs;
    shape.root = root;
    shape.np = np;
    shape.density = density;
    shape.K = K;
    shape.n_obs = D.n_obs;
    shape.precision = D.precision;
    shape.nonflat = K > 1 && n_nonroot == K && !flat_struct;
    std::string log;
    DeviceGuard guard(D.device);
    found = rtc_variant(shape, D.device, &st, &log);
    if (!found) {
      if (!log.empty()) std::fprintf(stderr, "nllmi: run-time compilation failed:\n%s\n", log.c_str());
      return st != NLL_OK ? st : NLL_ERR_DEVICE;
    }
    perm.resize(L);
    for (int l = 0; l < L; ++l) perm[l] = l;
  }

  std::memset(&pl, 0, sizeof(pl));
  pl.n_obs = D.n_obs;
  for (int o = 0; o < D.n_obs; ++o) {
    pl.lo[o] = D.obs_lo[o];
    pl.hi[o] = D.obs_hi[o];
  }
  pl.n_param = D.n_param;
  for (int k = 0; k < D.n_param; ++k) {
    pl.par_lo[k] = D.param_lo[k];
    pl.par_hi[k] = D.param_hi[k];
    pl.par_free[k] = D.param_free ? (D.param_free[k] ? 1 : 0) : 1;
  }
  std::vector<int> slot_of(L);
  pl.n_leaf = L;
  for (int s = 0; s < L; ++s) {
    const int l = perm[s];
    slot_of[l] = s;
    const nll_node_desc& nd = D.nodes[lw.leaves[l]];
    pl.leaf_kind[s] = nd.kind;
    pl.leaf_obs[s] = nd.obs;
    pl.leaf_np[s] = nd.n_param;
    for (int p = 0; p < nd.n_param; ++p) pl.leaf_param[s][p] = nd.param[p];
    pl.leaf_norm[s] = (nd.kind == NLL_HYPATIA || nd.kind == NLL_JIT) ? kNormGL : nd.norm;  // no closed form
    pl.leaf_root[s] = root[l];
  }
  // Flat shapes: term k is the one whose only non-root leaf sits in the
  // k-th non-root slot.
  if (flat_struct) {
    std::vector<Term> ordered;
    for (int sidx = 0; sidx < L; ++sidx) {
      const int l = perm[sidx];
      if (!root[l]) ordered.push_back(terms[term_of_leaf[l]]);
    }
    terms.swap(ordered);
  }
  pl.n_term = K;
  for (int k = 0; k < K; ++k) {
    uint32_t m = 0;
    for (int l = 0; l < L; ++l)
      if (((terms[k].mask >> l) & 1u) && !root[l]) m |= 1u << slot_of[l];
    pl.term_mask[k] = (int32_t)m;
    pl.term_nref[k] = (int32_t)terms[k].refs.size();
    for (size_t r = 0; r < terms[k].refs.size(); ++r) {
      pl.term_ref_sum[k][r] = terms[k].refs[r].first;
      pl.term_ref_child[k][r] = terms[k].refs[r].second;
    }
  }
  pl.n_sum = (int)lw.sums.size();
  for (int q = 0; q < pl.n_sum; ++q) {
    const nll_node_desc& nd = D.nodes[lw.sums[q]];
    pl.sum_nchild[q] = nd.n_child;
    pl.sum_yields[q] = nd.n_param == nd.n_child ? 1 : 0;
    for (int j = 0; j < nd.n_param; ++j) pl.sum_param[q][j] = nd.param[j];
  }
  // the expected count of an extended model without a yield parameter: the
  // root's sum of yields, or the one sum of yields among a root product's
  // children
  pl.ext_sum = -1;
  if (D.extended && D.yield_param < 0) {
    auto yields_pos = [&](int node) {
      const nll_node_desc& nd = D.nodes[node];
      return (nd.kind == NLL_SUM && nd.n_param == nd.n_child) ? lw.sum_pos[node] : -1;
    };
    const nll_node_desc& r = D.nodes[D.root];
    int found_sum = yields_pos(D.root), count = found_sum >= 0 ? 1 : 0;
    if (r.kind == NLL_PROD)
      for (int j = 0; j < r.n_child; ++j) {
        const int q = yields_pos(r.child[j]);
        if (q >= 0) {
          found_sum = q;
          ++count;
        }
      }
    if (count != 1) return NLL_ERR_ARG;
    pl.ext_sum = found_sum;
  }
  pl.acc_term_base = 1;
  int base = 1 + (K > 1 ? K : 0);
  for (int s = 0; s < L; ++s) {
    pl.acc_leaf_base[s] = base;
    base += pl.leaf_np[s];
  }
  pl.n_acc = found->na_grad;
  pl.extended = D.extended ? 1 : 0;
  pl.yield_param = D.extended && D.yield_param >= 0 ? D.yield_param : 0;
  *ops_out = found;
  return NLL_OK;
}

int tile_events(const nll_model* m) { return m->sched.unroll * kBlock; }

// the batched pass's chunks for the attached data and the current schedule
ChunkGrid chunk_grid(const nll_model* m) {
  return make_chunk_grid(std::max<int64_t>(m->n, 0), std::max(1, m->n_cu * m->sched.sets_blocks_per_cu),
                         m->sched.tile_events);
}

int single_grid(const nll_model* m) {
  const int64_t tiles = m->n > 0 ? (m->n + tile_events(m) - 1) / tile_events(m) : 1;
  int64_t g = (int64_t)m->n_cu * m->sched.blocks_per_cu;
  if (g > tiles) g = tiles;
  return (int)std::max<int64_t>(1, g);
}

// per-set arrays for n_sets sets and room for `items` work items (default:
// the most that consecutive event ranges can need)
nll_status ensure_sets(nll_model* m, int n_sets, int64_t items = -1) {
  if (n_sets > m->sets_cap) {
    dfree(m->tile_off);
    dfree(m->set_flag);
    dfree(m->consts);
    dfree(m->aux);
    m->sets_cap = 0;
    int cap = std::max(n_sets, 64);
    nll_status st;
    if ((st = dalloc(&m->tile_off, (size_t)cap + 1)) != NLL_OK) return st;
    if ((st = dalloc(&m->set_flag, (size_t)cap)) != NLL_OK) return st;
    if ((st = dalloc(&m->consts, (size_t)cap)) != NLL_OK) return st;
    if (m->ops->aux && (st = dalloc(&m->aux, (size_t)cap * kAuxWords)) != NLL_OK) return st;
    m->sets_cap = cap;
    m->have_graph = false;
  }
  // work items: the parts of the sets in the chunks of the batched pass (a
  // set's part per chunk it meets, at least one per set): at most
  // n_sets + chunks
  const ChunkGrid g = chunk_grid(m);
  const size_t chunks = (size_t)g.G * (size_t)g.K;
  if (items < 0) items = (int64_t)n_sets + (int64_t)chunks + 1;
  if (chunks + 1 > m->chunk_cap) {
    dfree(m->chunk_first);
    m->chunk_cap = 0;
    nll_status st = dalloc(&m->chunk_first, chunks + 1);
    if (st != NLL_OK) return st;
    m->chunk_cap = chunks + 1;
    m->have_graph = false;
  }
  if ((size_t)items > m->items_cap) {
    dfree(m->items);
    m->items_cap = 0;
    nll_status st = dalloc(&m->items, (size_t)items);
    if (st != NLL_OK) return st;
    m->items_cap = (size_t)items;
    m->have_graph = false;
  }
  const size_t need = (size_t)items * (size_t)(m->ops->na_grad + 1) * 2 * sizeof(double);
  if (need > m->set_partials_cap) {
    dfree(m->set_partials);
    m->set_partials_cap = 0;
    nll_status st = dalloc(reinterpret_cast<char**>(&m->set_partials), need);
    if (st != NLL_OK) return st;
    m->set_partials_cap = need;
    m->have_graph = false;
  }
  return NLL_OK;
}

nll_status ensure_gd(nll_model* m, int n_sets) {
  if (n_sets <= m->gd_cap) return NLL_OK;
  dfree(m->gd_mem);
  dfree(m->gd_status);
  dfree(m->gd_bacc);
  m->gd_cap = 0;
  const size_t P = (size_t)m->plan.n_param;
  nll_status st;
  if ((st = dalloc(&m->gd_mem, (size_t)n_sets * (3 * P + 2))) != NLL_OK) return st;
  if ((st = dalloc(&m->gd_status, (size_t)n_sets)) != NLL_OK) return st;
  if ((st = dalloc(&m->gd_bacc, (size_t)n_sets * P * P)) != NLL_OK) return st;
  m->gd_cap = n_sets;
  m->have_graph = false;
  return NLL_OK;
}

GDState gd_state(const nll_model* m) {
  const size_t P = (size_t)m->plan.n_param, S = (size_t)m->gd_cap;
  GDState g;
  g.th_acc = m->gd_mem;
  g.g_acc = m->gd_mem + S * P;
  g.th_prop = m->gd_mem + 2 * S * P;
  g.f_acc = m->gd_mem + 3 * S * P;
  g.eta = m->gd_mem + 3 * S * P + S;
  g.last_status = m->gd_status;
  g.b_acc = m->gd_bacc;
  return g;
}

SetsArgs sets_args(const nll_model* m, int n_sets, const int64_t* offsets) {
  SetsArgs a{};
  for (int o = 0; o < kMaxObs; ++o) a.cols[o] = m->cols[o];
  a.n_sets = n_sets;
  a.offsets = offsets;
  a.tile = m->sched.tile_events;
  a.tile_off = m->tile_off;
  a.set_flag = m->set_flag;
  a.items = m->items;
  a.chunk_first = m->chunk_first;
  a.rounds = chunk_grid(m).K;
  a.consts = m->consts;
  a.aux = m->aux;
  a.partials = m->set_partials;
  a.glx = m->gl.x;
  a.glw = m->gl.w;
  return a;
}

int sets_grid(const nll_model* m) { return std::max(1, m->n_cu * m->sched.sets_blocks_per_cu); }

// LDS per block that lets at most bpc blocks of the persistent grid share a
// CU (the dispatcher would otherwise pack up to the register limit onto
// some CUs and leave others short); 0 where no cap is needed or possible.
int lds_cap(const nll_model* m, int bpc) {
  if (bpc <= 0 || bpc >= 8 || m->lds_per_cu <= 0) return 0;
  const int cap = m->lds_per_cu / bpc - 256;
  return std::min(cap, m->lds_per_block);
}

SingleArgs single_args(const nll_model* m, const double* theta, double* nll_out, double* grad_out) {
  SingleArgs a{};
  for (int o = 0; o < kMaxObs; ++o) a.cols[o] = m->cols[o];
  if (m->weights) a.cols[m->plan.n_obs] = m->weights;  // read after the observables
  a.wsum = m->wsum;
  a.n = m->n;
  a.theta = theta;
  a.nll_out = nll_out;
  a.grad_out = grad_out;
  a.partials = m->partials;
  a.pt_out = m->pt_single;
  a.consts = m->consts;
  a.aux = m->aux;  // beside consts[0]: a fit's first step and BHHH steps
  a.status = m->status;
  a.glx = m->gl.x;
  a.glw = m->gl.w;
  return a;
}

// (re)create the step events of a timed fit
nll_status ensure_events(nll_model* m, int n_steps) {
  if (!m->step_timing) return NLL_OK;
  const int need = m->step_timing == 2 ? 2 * n_steps : n_steps + 1;
  while ((int)m->events.size() < need) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return NLL_ERR_DEVICE;
    m->events.push_back(e);
    m->have_graph = false;
  }
  return NLL_OK;
}

void record_step(nll_model* m, int s, hipStream_t st) {
  if (m->step_timing == 1) (void)hipEventRecord(m->events[s], st);
}

// start and stop events attached to the streaming kernel of step s
// (kernel timing only)
hipEvent_t kernel_event(nll_model* m, int s, int which) {
  return m->step_timing == 2 ? m->events[2 * s + which] : nullptr;
}

// the state of set `set` of the gradient-descent arrays, as a set-0 view
GDState gd_view(const GDState& g, int set, int P) {
  GDState v = g;
  v.th_acc += (size_t)set * P;
  v.g_acc += (size_t)set * P;
  v.th_prop += (size_t)set * P;
  v.f_acc += set;
  v.eta += set;
  v.last_status += set;
  if (v.b_acc) v.b_acc += (size_t)set * P * P;
  return v;
}

// a whole single-dataset fit.  Gradient descent: one launch per step, each
// taking the previous step's update before its pass (state, constants and
// block records alternate between two buffers by step parity; sets 0 and 1
// of the state arrays, constants 0 and 1, the two halves of the partials),
// and one finishing kernel for the last step's update.  BHHH: a streaming
// launch and a finishing kernel per step.
nll_status enqueue_fit_single(nll_model* m, hipStream_t st, double* theta, int n_steps, double eta, double* nll_out,
                              double* grad_out, int32_t* status_out, bool bhhh = false) {
  GDState gd = gd_state(m);
  hipError_t e = m->ops->fit_init(*m->ops, m->plan, theta, 1, eta, gd, m->consts, m->aux, m->gl.x, m->gl.w, st);
  if (e != hipSuccess) return NLL_ERR_DEVICE;
  SingleArgs a = single_args(m, nullptr, nullptr, nullptr);
  a.gd = gd;
  record_step(m, 0, st);
  const int grid = single_grid(m);
  const int cap = lds_cap(m, m->sched.blocks_per_cu);
  if (bhhh) {
    for (int s = 0; s < n_steps; ++s) {
      e = m->ops->single_bhhh_fit(*m->ops, m->plan, a, m->sched.unroll, grid, cap, st, kernel_event(m, s, 0),
                                  kernel_event(m, s, 1));
      if (e != hipSuccess) return NLL_ERR_DEVICE;
      record_step(m, s + 1, st);
    }
    e = launch_fit_final(1, m->plan.n_param, gd, theta, nll_out, grad_out, reinterpret_cast<int*>(status_out), st);
    return e == hipSuccess ? NLL_OK : NLL_ERR_DEVICE;
  }
  const int P = m->plan.n_param;
  const GDState gs[2] = {gd_view(gd, 0, P), gd_view(gd, 1, P)};
  double* part[2] = {m->partials, m->partials + m->partials_half};
  const auto step_fn = m->weights ? m->ops->single_w_fit : m->ops->single_fit;
  for (int s = 0; s < n_steps; ++s) {
    const int cur = s & 1, prev = cur ^ 1;
    a.partials = part[cur];
    a.partials_prev = s > 0 ? part[prev] : nullptr;
    a.gd = gs[prev];
    a.gd_out = gs[cur];
    a.consts = m->consts + (s > 0 ? prev : 0);
    a.consts_out = m->consts + cur;
    e = step_fn(*m->ops, m->plan, a, m->sched.unroll, grid, cap, st, kernel_event(m, s, 0), kernel_event(m, s, 1));
    if (e != hipSuccess) return NLL_ERR_DEVICE;
    if (s + 1 < n_steps) record_step(m, s + 1, st);  // the last step ends after its update
  }
  int last = 0;  // the buffer holding the final state
  if (n_steps > 0) {
    const int prev = (n_steps - 1) & 1;
    last = n_steps & 1;
    a.partials = part[prev];
    a.partials_prev = nullptr;
    a.gd = gs[prev];
    a.gd_out = gs[last];
    a.consts = m->consts + prev;
    a.consts_out = nullptr;
    e = (m->weights ? m->ops->w_fit_finish : m->ops->fit_finish)(*m->ops, m->plan, a, grid, st);
    if (e != hipSuccess) return NLL_ERR_DEVICE;
    record_step(m, n_steps, st);
  }
  e = launch_fit_final(1, P, gs[last], theta, nll_out, grad_out, reinterpret_cast<int*>(status_out), st);
  return e == hipSuccess ? NLL_OK : NLL_ERR_DEVICE;
}

// enqueue a whole fit on stream st
nll_status enqueue_fit(nll_model* m, hipStream_t st, int n_sets, const int64_t* offsets, double* theta,
                       int n_steps, double eta, double* nll_out, double* grad_out, int32_t* status_out) {
  GDState gd = gd_state(m);
  SetsArgs a = sets_args(m, n_sets, offsets);
  a.gd = gd;
  hipError_t e = launch_schedule(offsets, n_sets, chunk_grid(m), m->tile_off, m->set_flag, m->items,
                                 m->chunk_first, st);
  if (e != hipSuccess) return NLL_ERR_DEVICE;
  e = m->ops->fit_init(*m->ops, m->plan, theta, n_sets, eta, gd, m->consts, m->aux, m->gl.x, m->gl.w, st);
  if (e != hipSuccess) return NLL_ERR_DEVICE;
  record_step(m, 0, st);
  for (int s = 0; s < n_steps; ++s) {
    e = m->ops->sets(*m->ops, m->plan, a, true, true, m->sched.sets_unroll, sets_grid(m), lds_cap(m, m->sched.sets_blocks_per_cu),
                     st, kernel_event(m, s, 0), kernel_event(m, s, 1));
    if (e != hipSuccess) return NLL_ERR_DEVICE;
    record_step(m, s + 1, st);
  }
  e = launch_fit_final(n_sets, m->plan.n_param, gd, theta, nll_out, grad_out, reinterpret_cast<int*>(status_out), st);
  return e == hipSuccess ? NLL_OK : NLL_ERR_DEVICE;
}

// Enqueue through the model's recorded graph: capture once per argument
// set on the library's own stream, replay on the model's stream.
// Step timing runs eagerly: events recorded as nodes of a captured graph do
// not yield elapsed times.
template <class F>
nll_status run_recorded(nll_model* m, const FitKey& k, F&& enqueue) {
  if (!m->use_graph || m->step_timing) return enqueue(m->stream);
  if (!(m->have_graph && m->key == k)) {
    if (m->exec) (void)hipGraphExecDestroy(m->exec);
    if (m->graph) (void)hipGraphDestroy(m->graph);
    m->exec = nullptr;
    m->graph = nullptr;
    m->have_graph = false;
    if (hipStreamBeginCapture(m->capture, hipStreamCaptureModeThreadLocal) != hipSuccess) return NLL_ERR_DEVICE;
    nll_status est = enqueue(m->capture);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(m->capture, &g);
    if (est != NLL_OK || e != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return est != NLL_OK ? est : NLL_ERR_DEVICE;
    }
    if (hipGraphInstantiate(&m->exec, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(g);
      return NLL_ERR_DEVICE;
    }
    m->graph = g;
    m->key = k;
    m->have_graph = true;
  }
  return hipGraphLaunch(m->exec, m->stream) == hipSuccess ? NLL_OK : NLL_ERR_DEVICE;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
namespace nllmi {

nll_status batched_args_ok(const nll_model* m, int32_t n_sets, const int64_t* offsets, const double* theta,
                           const double* nll_out) {
  if (!m || n_sets < 0 || (n_sets > 0 && (!offsets || !theta || !nll_out))) return NLL_ERR_ARG;
  if (m->n < 0) return NLL_ERR_STATE;
  if (m->weights) return NLL_ERR_UNSUPPORTED;
  return NLL_OK;
}

int64_t batched_items_bound(const nll_model* m, int32_t n_sets) {
  const ChunkGrid g = chunk_grid(m);
  return (int64_t)n_sets + (int64_t)g.G * g.K + 1;
}

size_t batched_record_bytes(const nll_model* m) { return (size_t)(m->ops->na_grad + 1) * 2 * sizeof(double); }

nll_status eval_batched_on(nll_model* m, int32_t n_sets, const int64_t* offsets, const double* theta,
                           double* nll_out, double* grad_out, int32_t* status_out, const SetsScratch& s) {
  const bool grad = grad_out != nullptr;
  SetsArgs a = sets_args(m, n_sets, offsets);
  a.tile_off = s.tile_off;
  a.set_flag = s.set_flag;
  a.items = s.items;
  a.chunk_first = s.chunk_first;
  a.consts = s.consts;
  a.aux = s.aux;
  a.partials = s.partials;
  a.theta = theta;
  a.nll_out = nll_out;
  a.grad_out = grad_out;
  a.status_out = reinterpret_cast<int*>(status_out);
  if (launch_schedule(offsets, n_sets, chunk_grid(m), s.tile_off, s.set_flag, s.items, s.chunk_first,
                      m->stream) !=
      hipSuccess)
    return NLL_ERR_DEVICE;
  if (m->ops->consts(*m->ops, m->plan, theta, n_sets, s.consts, s.aux, m->gl.x, m->gl.w, m->stream) != hipSuccess)
    return NLL_ERR_DEVICE;
  if (m->ops->sets(*m->ops, m->plan, a, grad, false, m->sched.sets_unroll, sets_grid(m), lds_cap(m, m->sched.sets_blocks_per_cu),
                   m->stream, nullptr, nullptr) != hipSuccess)
    return NLL_ERR_DEVICE;
  return NLL_OK;
}

}  // namespace nllmi

extern "C" {

const char* nll_status_string(nll_status s) {
  switch (s) {
    case NLL_OK: return "ok";
    case NLL_ERR_ARG: return "invalid argument";
    case NLL_ERR_UNSUPPORTED: return "model shape not supported by the compiled kernels";
    case NLL_ERR_PARAM_RANGE: return "parameter outside its allowed range";
    case NLL_ERR_DOMAIN: return "event outside the observable range";
    case NLL_ERR_INVALID_PDF: return "probability density <= 0 or not finite";
    case NLL_ERR_DEVICE: return "HIP runtime error";
    case NLL_ERR_OOM: return "out of device memory";
    case NLL_ERR_STATE: return "call out of order";
    case NLL_ERR_SCRATCH: return "request larger than the fixed scratch array of the no-allocation entry point";
  }
  return "unknown status";
}

nll_status nll_create_model(const nll_model_desc* desc, nll_model** out) {
  if (!desc || !out) return NLL_ERR_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return NLL_ERR_DEVICE;
  if (desc->device < 0 || desc->device >= ndev) return NLL_ERR_ARG;
  Plan pl;
  const VariantOps* ops = nullptr;
  nll_status st = build_plan(*desc, pl, &ops);
  if (st != NLL_OK) return st;

  DeviceGuard guard(desc->device);
  nll_model* m = new (std::nothrow) nll_model();
  if (!m) return NLL_ERR_OOM;
  m->device = desc->device;
  m->stream = reinterpret_cast<hipStream_t>(desc->stream);
  m->plan = pl;
  m->ops = ops;
  m->precision = desc->precision;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, desc->device) == hipSuccess && cus > 0)
    m->n_cu = cus;
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, desc->device) == hipSuccess)
    m->lds_per_cu = lds;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, desc->device) == hipSuccess)
    m->lds_per_block = lds;
  auto fail = [&](nll_status s) {
    nll_destroy_model(m);
    return s;
  };
  // shapes with many gradient accumulators keep 2 events per thread per
  // tile (4 interleaved events exceed the register file: measured slower)
  if (ops->na_grad > 8) m->sched.unroll = 2;
  if ((st = gl_table(m->device, &m->gl)) != NLL_OK) return fail(st);
  const size_t max_grid = (size_t)m->n_cu * 32;
  const size_t record = std::max<size_t>((size_t)ops->na_grad + 1, (size_t)ops->bhhh_record);
  // two halves: gradient-descent steps alternate between them
  m->partials_half = max_grid * record * 2;
  if ((st = dalloc(&m->partials, 2 * m->partials_half)) != NLL_OK) return fail(st);
  if ((st = dalloc(&m->pt_single, 1)) != NLL_OK) return fail(st);
  if ((st = dalloc(&m->status, 1)) != NLL_OK) return fail(st);
  if ((st = dalloc(&m->dbad, 1)) != NLL_OK) return fail(st);
  if ((st = dalloc(&m->offsets1, 2)) != NLL_OK) return fail(st);
  if (hipMemset(m->status, 0, sizeof(int)) != hipSuccess)
    return fail(NLL_ERR_DEVICE);
  if (hipStreamCreateWithFlags(&m->capture, hipStreamNonBlocking) != hipSuccess) return fail(NLL_ERR_DEVICE);
  *out = m;
  return NLL_OK;
}

void nll_destroy_model(nll_model* m) {
  if (!m) return;
  DeviceGuard guard(m->device);
  (void)hipStreamSynchronize(m->stream);
  if (m->exec) (void)hipGraphExecDestroy(m->exec);
  if (m->graph) (void)hipGraphDestroy(m->graph);
  if (m->capture) (void)hipStreamDestroy(m->capture);
  for (hipEvent_t e : m->events) (void)hipEventDestroy(e);
  dfree(m->partials);
  dfree(m->pt_single);
  dfree(m->status);
  dfree(m->dbad);
  dfree(m->offsets1);
  dfree(m->pts_offsets);
  dfree(m->tile_off);
  dfree(m->set_flag);
  dfree(m->items);
  dfree(m->chunk_first);
  dfree(m->consts);
  dfree(m->aux);
  dfree(m->set_partials);
  dfree(m->gd_mem);
  dfree(m->gd_status);
  dfree(m->gd_bacc);
  dfree(m->wsum);
  dfree(m->wsum_part);
  delete m;
}

nll_status nll_set_stream(nll_model* m, void* stream) {
  if (!m) return NLL_ERR_ARG;
  m->stream = reinterpret_cast<hipStream_t>(stream);
  return NLL_OK;
}

nll_status nll_set_data(nll_model* m, const double* const* cols, int64_t n_events) {
  if (!m || n_events < 0 || (n_events > 0 && !cols)) return NLL_ERR_ARG;
  for (int o = 0; o < m->plan.n_obs && n_events > 0; ++o)
    if (!cols[o] || (reinterpret_cast<uintptr_t>(cols[o]) & 7u)) return NLL_ERR_ARG;
  DeviceGuard guard(m->device);
  unsigned long long bad = 0;
  for (int o = 0; o < m->plan.n_obs && n_events > 0; ++o) {
    if (hipMemsetAsync(m->dbad, 0, sizeof(unsigned long long), m->stream) != hipSuccess) return NLL_ERR_DEVICE;
    if (launch_check_range(cols[o], n_events, m->plan.lo[o], m->plan.hi[o], m->dbad, m->stream) != hipSuccess)
      return NLL_ERR_DEVICE;
    unsigned long long b = 0;
    if (hipMemcpyAsync(&b, m->dbad, sizeof(b), hipMemcpyDeviceToHost, m->stream) != hipSuccess ||
        hipStreamSynchronize(m->stream) != hipSuccess)
      return NLL_ERR_DEVICE;
    bad += b;
  }
  if (bad) return NLL_ERR_DOMAIN;
  for (int o = 0; o < kMaxObs; ++o) m->cols[o] = (o < m->plan.n_obs && n_events > 0) ? cols[o] : nullptr;
  m->n = n_events;
  m->weights = nullptr;  // weights belong to the data they were attached to
  const int64_t off[2] = {0, n_events};
  if (hipMemcpy(m->offsets1, off, sizeof(off), hipMemcpyHostToDevice) != hipSuccess) return NLL_ERR_DEVICE;
  m->have_graph = false;
  return NLL_OK;
}

nll_status nll_set_weights(nll_model* m, const double* weights) {
  if (!m) return NLL_ERR_ARG;
  if (m->n < 0) return NLL_ERR_STATE;
  if (weights && (reinterpret_cast<uintptr_t>(weights) & 7u)) return NLL_ERR_ARG;
  if (weights && !m->ops->single_w) return NLL_ERR_UNSUPPORTED;
  DeviceGuard guard(m->device);
  m->weights = nullptr;
  m->have_graph = false;
  if (!weights || m->n == 0) return NLL_OK;
  nll_status st = NLL_OK;
  if (!m->wsum && (st = dalloc(&m->wsum, 1)) != NLL_OK) return st;
  if (!m->wsum_part && (st = dalloc(&m->wsum_part, 2 * (size_t)kWsumBlocks)) != NLL_OK) return st;
  // W once per attachment, on the model's stream (ahead of every use)
  if (launch_wsum(weights, m->n, m->wsum_part, m->wsum, m->stream) != hipSuccess) return NLL_ERR_DEVICE;
  m->weights = weights;
  return NLL_OK;
}

static nll_status nll_eval_impl(nll_model* m, const double* theta, double* nll_out, double* grad_out, bool grad) {
  if (!m || !theta || !nll_out || (grad && !grad_out)) return NLL_ERR_ARG;
  if (m->n < 0) return NLL_ERR_STATE;
  DeviceGuard guard(m->device);
  SingleArgs a = single_args(m, theta, nll_out, grad_out);
  hipError_t e = (m->weights ? m->ops->single_w : m->ops->single)(
      *m->ops, m->plan, a, grad, m->sched.unroll, single_grid(m), lds_cap(m, m->sched.blocks_per_cu), m->stream);
  return e == hipSuccess ? NLL_OK : NLL_ERR_DEVICE;
}

nll_status nll_eval_bhhh(nll_model* m, const double* theta, double* nll_out, double* grad_out, double* bhhh_out) {
  if (!m || !theta || !nll_out || !grad_out || !bhhh_out) return NLL_ERR_ARG;
  if (!m->ops->single_bhhh || m->weights) return NLL_ERR_UNSUPPORTED;
  if (m->n < 0) return NLL_ERR_STATE;
  DeviceGuard guard(m->device);
  SingleArgs a = single_args(m, theta, nll_out, grad_out);
  a.bhhh_out = bhhh_out;
  hipError_t e = m->ops->single_bhhh(*m->ops, m->plan, a, m->sched.unroll, single_grid(m), lds_cap(m, m->sched.blocks_per_cu),
                                     m->stream);
  return e == hipSuccess ? NLL_OK : NLL_ERR_DEVICE;
}

nll_status nll_eval(nll_model* m, const double* theta, double* nll_out) {
  return nll_eval_impl(m, theta, nll_out, nullptr, false);
}

nll_status nll_eval_grad(nll_model* m, const double* theta, double* nll_out, double* grad_out) {
  return nll_eval_impl(m, theta, nll_out, grad_out, true);
}

nll_status nll_eval_batched(nll_model* m, int32_t n_sets, const int64_t* offsets, const double* theta,
                            double* nll_out, double* grad_out, int32_t* status_out) {
  nll_status st = batched_args_ok(m, n_sets, offsets, theta, nll_out);
  if (st != NLL_OK || n_sets == 0) return st;
  DeviceGuard guard(m->device);
  if ((st = ensure_sets(m, n_sets)) != NLL_OK) return st;
  SetsScratch s;
  s.tile_off = m->tile_off;
  s.chunk_first = m->chunk_first;
  s.set_flag = m->set_flag;
  s.items = m->items;
  s.consts = m->consts;
  s.aux = m->aux;
  s.partials = m->set_partials;
  return eval_batched_on(m, n_sets, offsets, theta, nll_out, grad_out, status_out, s);
}

nll_status nll_eval_points(nll_model* m, int32_t n_points, const double* theta, double* nll_out, double* grad_out,
                           int32_t* status_out) {
  if (!m || n_points < 0 || (n_points > 0 && (!theta || !nll_out))) return NLL_ERR_ARG;
  if (m->n < 0) return NLL_ERR_STATE;
  if (m->weights) return NLL_ERR_UNSUPPORTED;
  if (n_points == 0) return NLL_OK;
  DeviceGuard guard(m->device);
  // The (point, tile) work items of a small dataset would leave most of a
  // grid of the batched pass idle while a few blocks run long chains of
  // tiles: the model's tile is halved (down to 4096 events, keeping a
  // multiple of 512) until there are two items per block of a grid of at
  // most 4 blocks per CU (1e5 events x 64 points: 16384 -> 4096 events,
  // 41 -> 23 us measured).
  const int bpc = std::min(m->sched.sets_blocks_per_cu, 4);
  const int grid = std::max(1, m->n_cu * bpc);
  int64_t tile = m->sched.tile_events;
  auto items = [&](int64_t t) { return (int64_t)n_points * (m->n > 0 ? (m->n + t - 1) / t : 1); };
  while (tile / 2 >= 4096 && (tile / 2) % 512 == 0 && items(tile) < 2 * (int64_t)grid) tile /= 2;
  const int64_t per = m->n > 0 ? (m->n + tile - 1) / tile : 1;
  nll_status st = ensure_sets(m, n_points, (int64_t)n_points * per);
  if (st != NLL_OK) return st;
  if (n_points > m->pts_cap) {
    dfree(m->pts_offsets);
    m->pts_cap = 0;
    if ((st = dalloc(&m->pts_offsets, (size_t)n_points + 1)) != NLL_OK) return st;
    m->pts_cap = n_points;
  }
  SetsArgs a = sets_args(m, n_points, m->pts_offsets);
  a.theta = theta;
  a.nll_out = nll_out;
  a.grad_out = grad_out;
  a.status_out = reinterpret_cast<int*>(status_out);
  a.rounds = 1;  // points: one round of G chunks of equal item counts
  a.tile = tile;
  if (launch_points(n_points, m->n, tile, grid, m->pts_offsets, m->tile_off, m->set_flag, m->items,
                    m->chunk_first, m->stream) != hipSuccess)
    return NLL_ERR_DEVICE;
  if (m->ops->consts(*m->ops, m->plan, theta, n_points, m->consts, m->aux, m->gl.x, m->gl.w, m->stream) != hipSuccess)
    return NLL_ERR_DEVICE;
  if (m->ops->sets(*m->ops, m->plan, a, grad_out != nullptr, false, m->sched.sets_unroll, grid, lds_cap(m, bpc),
                   m->stream, nullptr, nullptr) != hipSuccess)
    return NLL_ERR_DEVICE;
  return NLL_OK;
}

nll_status nll_fit_batched(nll_model* m, int32_t n_sets, const int64_t* offsets, double* theta, int32_t n_steps,
                           double eta, double* nll_out, double* grad_out, int32_t* status_out) {
  if (!m || n_sets < 0 || n_steps < 0 || !(eta > 0.0) || (n_sets > 0 && (!offsets || !theta || !nll_out)))
    return NLL_ERR_ARG;
  if (m->n < 0) return NLL_ERR_STATE;
  if (m->weights) return NLL_ERR_UNSUPPORTED;
  if (n_sets == 0) return NLL_OK;
  DeviceGuard guard(m->device);
  nll_status st = ensure_sets(m, n_sets);
  if (st != NLL_OK) return st;
  if ((st = ensure_gd(m, n_sets)) != NLL_OK) return st;
  FitKey k;
  k.mode = 2;
  k.timing = m->step_timing;
  if ((st = ensure_events(m, n_steps)) != NLL_OK) return st;
  m->timed_steps = m->step_timing ? n_steps : -1;
  m->timed_mode = m->step_timing;
  k.n_sets = n_sets;
  k.offsets = offsets;
  k.theta = theta;
  k.n_steps = n_steps;
  k.eta = eta;
  k.nll = nll_out;
  k.grad = grad_out;
  k.status = status_out;
  k.sched = m->sched;
  return run_recorded(m, k, [&](hipStream_t st) {
    return enqueue_fit(m, st, n_sets, offsets, theta, n_steps, eta, nll_out, grad_out, status_out);
  });
}

static nll_status fit_single_impl(nll_model* m, double* theta, int32_t n_steps, double eta, double* nll_out,
                                  double* grad_out, int32_t* status_out, bool bhhh) {
  if (!m || !theta || !nll_out || n_steps < 0 || !(eta > 0.0)) return NLL_ERR_ARG;
  if (bhhh && (!m->ops->single_bhhh_fit || m->weights)) return NLL_ERR_UNSUPPORTED;
  if (m->n < 0) return NLL_ERR_STATE;
  DeviceGuard guard(m->device);
  nll_status st = ensure_sets(m, 1);
  if (st != NLL_OK) return st;
  if ((st = ensure_gd(m, 2)) != NLL_OK) return st;  // gradient descent: two state buffers
  FitKey k;
  k.mode = bhhh ? 3 : 1;
  k.timing = m->step_timing;
  if ((st = ensure_events(m, n_steps)) != NLL_OK) return st;
  m->timed_steps = m->step_timing ? n_steps : -1;
  m->timed_mode = m->step_timing;
  k.n_sets = 1;
  k.theta = theta;
  k.n_steps = n_steps;
  k.eta = eta;
  k.nll = nll_out;
  k.grad = grad_out;
  k.status = status_out;
  k.sched = m->sched;
  return run_recorded(m, k, [&](hipStream_t s) {
    return enqueue_fit_single(m, s, theta, n_steps, eta, nll_out, grad_out, status_out, bhhh);
  });
}

nll_status nll_fit(nll_model* m, double* theta, int32_t n_steps, double eta, double* nll_out, double* grad_out,
                   int32_t* status_out) {
  return fit_single_impl(m, theta, n_steps, eta, nll_out, grad_out, status_out, false);
}

nll_status nll_fit_bhhh(nll_model* m, double* theta, int32_t n_steps, double lambda, double* nll_out,
                        double* grad_out, int32_t* status_out) {
  return fit_single_impl(m, theta, n_steps, lambda, nll_out, grad_out, status_out, true);
}

nll_status nll_sync(nll_model* m, int32_t* status_out) {
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
  return st;
}

nll_status nll_get_schedule(const nll_model* m, nll_schedule* out) {
  if (!m || !out) return NLL_ERR_ARG;
  *out = m->sched;
  return NLL_OK;
}

nll_status nll_set_schedule(nll_model* m, const nll_schedule* s) {
  if (!m || !s) return NLL_ERR_ARG;
  auto valid_u = [](int u) { return u == 2 || u == 4 || u == 8; };
  if (!valid_u(s->unroll) || !valid_u(s->sets_unroll)) return NLL_ERR_ARG;
  if (s->blocks_per_cu < 1 || s->blocks_per_cu > 32) return NLL_ERR_ARG;
  if (s->tile_events < 1024 || s->tile_events > (1 << 22) || (s->tile_events % 512) != 0) return NLL_ERR_ARG;
  if (s->sets_blocks_per_cu < 1 || s->sets_blocks_per_cu > 32) return NLL_ERR_ARG;
  if (std::memcmp(&m->sched, s, sizeof(*s)) != 0) m->have_graph = false;
  m->sched = *s;
  return NLL_OK;
}

nll_status nll_autotune(nll_model* m, int32_t which, int32_t n_sets, const int64_t* offsets, const double* theta) {
  if (!m || (which != 1 && which != 2)) return NLL_ERR_ARG;
  if (m->n < 0) return NLL_ERR_STATE;
  if (m->weights) return NLL_ERR_UNSUPPORTED;
  DeviceGuard guard(m->device);
  return tune_model(m, which, n_sets, offsets, theta);
}

nll_status nll_set_option(nll_model* m, int32_t option, int32_t value) {
  if (!m) return NLL_ERR_ARG;
  if (option == NLL_OPT_GRAPH) {
    m->use_graph = value != 0;
  } else if (option == NLL_OPT_STEP_TIMING) {
    if (value < 0 || value > 2) return NLL_ERR_ARG;
    m->step_timing = value;
  } else {
    return NLL_ERR_ARG;
  }
  m->have_graph = false;
  return NLL_OK;
}

nll_status nll_step_times(nll_model* m, float* ms, int32_t cap, int32_t* n) {
  if (!m || !n || cap < 0 || (cap > 0 && !ms)) return NLL_ERR_ARG;
  if (m->timed_steps < 0) return NLL_ERR_STATE;
  DeviceGuard guard(m->device);
  if (hipStreamSynchronize(m->stream) != hipSuccess) return NLL_ERR_DEVICE;
  const int k = std::min(cap, m->timed_steps);
  for (int s = 0; s < k; ++s) {
    const hipEvent_t a = m->timed_mode == 2 ? m->events[2 * s] : m->events[s];
    const hipEvent_t b = m->timed_mode == 2 ? m->events[2 * s + 1] : m->events[s + 1];
    if (hipEventElapsedTime(&ms[s], a, b) != hipSuccess) return NLL_ERR_DEVICE;
  }
  *n = k;
  return NLL_OK;
}

nll_status nll_read_probe(const double* x, int64_t n, double* block_sums, int32_t n_blocks, void* stream) {
  if (!x || !block_sums || n < 0 || n_blocks < 1 || n_blocks > (1 << 20)) return NLL_ERR_ARG;
  if ((reinterpret_cast<uintptr_t>(x) & 15u) != 0) return NLL_ERR_ARG;
  return launch_read_probe(x, n, block_sums, n_blocks, static_cast<hipStream_t>(stream)) == hipSuccess
             ? NLL_OK
             : NLL_ERR_DEVICE;
}

nll_status nll_get_info(const nll_model* m, nll_info* out) {
  if (!m || !out) return NLL_ERR_ARG;
  std::memset(out, 0, sizeof(*out));
  std::strncpy(out->variant, m->ops->name, sizeof(out->variant) - 1);
  out->n_leaf = m->plan.n_leaf;
  out->n_term = m->plan.n_term;
  out->n_accumulators = m->ops->na_grad;
  out->precision = m->precision;
  out->n_cu = m->n_cu;
  out->n_events = m->n;
  out->per_set_bytes = (int32_t)(sizeof(PerTheta) + (m->ops->aux ? kAuxWords * sizeof(double) : 0));
  return NLL_OK;
}

}  // extern "C"
