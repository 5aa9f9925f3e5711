// Kernels of dimension 4 (see kernels.h).
#include "kernels.h"

namespace pcms {
PCMS_DEFINE_DIM_KERNELS(4)
}  // namespace pcms
