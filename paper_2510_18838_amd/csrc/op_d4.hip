// Operator-emission kernels of dimension 4 (see kernels.h).
#include "kernels.h"

namespace pcms {
PCMS_DEFINE_DIM_OPERATOR(4)
}  // namespace pcms
