// Operator-emission kernels of dimension 3 (see kernels.h).
#include "kernels.h"

namespace pcms {
PCMS_DEFINE_DIM_OPERATOR(3)
}  // namespace pcms
