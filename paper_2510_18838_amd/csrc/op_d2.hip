// Operator-emission kernels of dimension 2 (see kernels.h).
#include "kernels.h"

namespace pcms {
PCMS_DEFINE_DIM_OPERATOR(2)
}  // namespace pcms
