// rtc.h -- model shapes outside the ahead-of-time registry, compiled at run
// time (hipRTC) from the same kernel templates.
#pragma once

#include <string>
#include <vector>

#include "kernels.h"
#include "nll.h"

namespace nllmi {

// A lowered shape: leaves in slot order (kind, observable, root factor,
// parameter count), K terms over n_obs observables, the precision of the
// event pass, and whether the plan's term masks rather than the slot order
// define the terms (a shape with as many non-root leaves as terms whose
// terms are not one non-root leaf each, e.g. a product of two sums).
struct RtcShape {
  std::vector<int> kind, obs, root, np;
  std::vector<std::string> density;  // per leaf: the formula of a formula leaf (kJit), else empty
  int K = 1, n_obs = 1, precision = 0;
  bool nonflat = false;
};

// The variant for `shape` on `device` (the current device): compiled on the
// first request in the process (or loaded from the on-disk code-object
// cache), kept until the process ends.  On failure returns null with
// *status set (NLL_ERR_DEVICE; the compiler's log in *log).
const VariantOps* rtc_variant(const RtcShape& shape, int device, nll_status* status, std::string* log);

// The type name of the model that rtc_variant compiles for `shape`.
std::string rtc_model_type(const RtcShape& shape);

// Compile `shape` for `arch` (e.g. "gfx950") without loading it: needs no
// device (a build-time check of the templates).  NLL_OK or NLL_ERR_DEVICE
// with the compiler's log.
nll_status rtc_compile_check(const RtcShape& shape, const std::string& arch, std::string* log);

}  // namespace nllmi
