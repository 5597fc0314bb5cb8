// variants_hypatia.hip -- compiled shapes with the Hypatia2 leaf: alone,
// and as the signal of a signal-plus-exponential mixture.  FP64 only (the
// leaf has no FP32-compensated form).
#include "kernels_impl.h"

namespace nllmi {

void register_variants_hypatia(std::vector<VariantOps>& out) {
  out.push_back(make_ops<Model<1, 1, Slot<HypatiaLeaf, 0, true>>>("hypatia"));
  out.push_back(make_ops<Model<2, 1, Slot<HypatiaLeaf, 0, false>, Slot<ExpLeaf, 0, false>>>("hypatia+exp"));
}

}  // namespace nllmi
