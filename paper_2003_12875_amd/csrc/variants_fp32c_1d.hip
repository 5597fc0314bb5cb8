// variants_fp32c_1d.hip -- the one-observable shapes with the
// FP32-compensated event pass.
#include "kernels_impl.h"

namespace nllmi {

void register_variants_fp32c_1d(std::vector<VariantOps>& out) {
  out.push_back(make_ops<FP32C<Model<1, 1, Slot<GaussLeaf, 0, true>>>>("gauss/fp32c"));
  out.push_back(make_ops<FP32C<Model<1, 1, Slot<ExpLeaf, 0, true>>>>("exp/fp32c"));
  out.push_back(make_ops<FP32C<Model<1, 1, Slot<CBLeaf, 0, true>>>>("cb/fp32c"));
  out.push_back(make_ops<FP32C<Model<1, 1, Slot<ArgusLeaf, 0, true>>>>("argus/fp32c"));
  out.push_back(make_ops<FP32C<Model<1, 1, Slot<ChebLeaf<2>, 0, true>>>>("cheb2/fp32c"));
  out.push_back(make_ops<FP32C<Model<1, 1, Slot<ChebLeaf<4>, 0, true>>>>("cheb4/fp32c"));
  out.push_back(make_ops<FP32C<Model<2, 1, Slot<GaussLeaf, 0, false>, Slot<ExpLeaf, 0, false>>>>("gauss+exp/fp32c"));
  out.push_back(
      make_ops<FP32C<Model<2, 1, Slot<GaussLeaf, 0, false>, Slot<GaussLeaf, 0, false>>>>("gauss+gauss/fp32c"));
  out.push_back(make_ops<FP32C<Model<2, 1, Slot<CBLeaf, 0, false>, Slot<ArgusLeaf, 0, false>>>>("cb+argus/fp32c"));
}

}  // namespace nllmi
