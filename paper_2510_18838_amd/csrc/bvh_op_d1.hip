// Operator-emission kernels of dimension 1 on an LBVH (see kernels.h).
#include "kernels.h"

namespace pcms {
PCMS_DEFINE_DIM_OPERATOR_BVH(1)
}  // namespace pcms
