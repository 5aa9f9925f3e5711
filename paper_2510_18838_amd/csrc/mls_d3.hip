// Kernels of dimension 3 (see kernels.h).
#include "kernels.h"

namespace pcms {
PCMS_DEFINE_DIM_KERNELS(3)
}  // namespace pcms
