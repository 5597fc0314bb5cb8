// variants_johnson.hip -- compiled shapes with the Johnson S_U leaf: alone
// and as the peak of a two-component mixture over an exponential
// background, each in FP64 and with the FP32-compensated event pass.
#include "kernels_impl.h"

namespace nllmi {

void register_variants_johnson(std::vector<VariantOps>& out) {
  out.push_back(make_ops<Model<1, 1, Slot<JohnsonLeaf, 0, true>>>("johnson"));
  out.push_back(make_ops<Model<2, 1, Slot<JohnsonLeaf, 0, false>, Slot<ExpLeaf, 0, false>>>("johnson+exp"));
  out.push_back(make_ops<FP32C<Model<1, 1, Slot<JohnsonLeaf, 0, true>>>>("johnson/fp32c"));
  out.push_back(
      make_ops<FP32C<Model<2, 1, Slot<JohnsonLeaf, 0, false>, Slot<ExpLeaf, 0, false>>>>("johnson+exp/fp32c"));
}

}  // namespace nllmi
