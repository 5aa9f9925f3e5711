// Kernels of dimension 2 (see kernels.h).
#include "kernels.h"

namespace pcms {
PCMS_DEFINE_DIM_KERNELS(2)
}  // namespace pcms
