// Kernels of dimension 5 on an LBVH (see kernels.h).
#include "kernels.h"

namespace pcms {
PCMS_DEFINE_DIM_BVH(5)
}  // namespace pcms
