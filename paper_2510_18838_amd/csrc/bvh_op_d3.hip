// Operator-emission kernels of dimension 3 on an LBVH (see kernels.h).
#include "kernels.h"

namespace pcms {
PCMS_DEFINE_DIM_OPERATOR_BVH(3)
}  // namespace pcms
