// Operator-emission kernels of dimension 4 on an LBVH (see kernels.h).
#include "kernels.h"

namespace pcms {
PCMS_DEFINE_DIM_OPERATOR_BVH(4)
}  // namespace pcms
