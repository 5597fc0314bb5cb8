// variants_2d.hip -- compiled shapes over two observables.
#include "kernels_impl.h"

namespace nllmi {

void register_variants_2d(std::vector<VariantOps>& out) {
  out.push_back(make_ops<Model<2, 2, Slot<CBLeaf, 0, false>, Slot<ArgusLeaf, 0, false>,
                               Slot<ChebLeaf<4>, 1, true>>>("(cb+argus)*cheb4"));
  out.push_back(make_ops<Model<1, 2, Slot<GaussLeaf, 0, true>, Slot<GaussLeaf, 1, true>>>("gauss*gauss"));
}

}  // namespace nllmi
