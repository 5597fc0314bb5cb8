// variants_mixture.hip -- compiled shapes: two-component mixtures on one
// observable.
#include "kernels_impl.h"

namespace nllmi {

void register_variants_mixture(std::vector<VariantOps>& out) {
  out.push_back(make_ops<Model<2, 1, Slot<GaussLeaf, 0, false>, Slot<ExpLeaf, 0, false>>>("gauss+exp"));
  out.push_back(make_ops<Model<2, 1, Slot<GaussLeaf, 0, false>, Slot<GaussLeaf, 0, false>>>("gauss+gauss"));
  out.push_back(make_ops<Model<2, 1, Slot<CBLeaf, 0, false>, Slot<ArgusLeaf, 0, false>>>("cb+argus"));
}

}  // namespace nllmi
