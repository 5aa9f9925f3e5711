// Kernels of dimension 2 on an LBVH (see kernels.h).
#include "kernels.h"

namespace pcms {
PCMS_DEFINE_DIM_BVH(2)
}  // namespace pcms
