// Operator-emission kernels of dimension 1 (see kernels.h).
#include "kernels.h"

namespace pcms {
PCMS_DEFINE_DIM_OPERATOR(1)
}  // namespace pcms
