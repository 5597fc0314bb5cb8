// variants_single.hip -- compiled shapes with one leaf (no mixture).
#include "kernels_impl.h"

namespace nllmi {

void register_variants_single(std::vector<VariantOps>& out) {
  out.push_back(make_ops<Model<1, 1, Slot<GaussLeaf, 0, true>>>("gauss"));
  out.push_back(make_ops<Model<1, 1, Slot<ExpLeaf, 0, true>>>("exp"));
  out.push_back(make_ops<Model<1, 1, Slot<CBLeaf, 0, true>>>("cb"));
  out.push_back(make_ops<Model<1, 1, Slot<ArgusLeaf, 0, true>>>("argus"));
  out.push_back(make_ops<Model<1, 1, Slot<ChebLeaf<2>, 0, true>>>("cheb2"));
  out.push_back(make_ops<Model<1, 1, Slot<ChebLeaf<4>, 0, true>>>("cheb4"));
}

}  // namespace nllmi
