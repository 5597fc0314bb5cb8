// variants_fp32c_2d.hip -- the two-observable shapes with the
// FP32-compensated event pass.
#include "kernels_impl.h"

namespace nllmi {

void register_variants_fp32c_2d(std::vector<VariantOps>& out) {
  out.push_back(make_ops<FP32C<Model<2, 2, Slot<CBLeaf, 0, false>, Slot<ArgusLeaf, 0, false>,
                                     Slot<ChebLeaf<4>, 1, true>>>>("(cb+argus)*cheb4/fp32c"));
  out.push_back(make_ops<FP32C<Model<1, 2, Slot<GaussLeaf, 0, true>, Slot<GaussLeaf, 1, true>>>>("gauss*gauss/fp32c"));
}

}  // namespace nllmi
