// variants_chi2.hip -- compiled shapes with the chi-square leaf alone, in
// FP64 and with the FP32-compensated event pass.
#include "kernels_impl.h"

namespace nllmi {

void register_variants_chi2(std::vector<VariantOps>& out) {
  out.push_back(make_ops<Model<1, 1, Slot<Chi2Leaf, 0, true>>>("chi2"));
  out.push_back(make_ops<FP32C<Model<1, 1, Slot<Chi2Leaf, 0, true>>>>("chi2/fp32c"));
}

}  // namespace nllmi
