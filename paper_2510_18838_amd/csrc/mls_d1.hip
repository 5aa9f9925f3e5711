// Kernels of dimension 1 (see kernels.h).
#include "kernels.h"

namespace pcms {
PCMS_DEFINE_DIM_KERNELS(1)
}  // namespace pcms
