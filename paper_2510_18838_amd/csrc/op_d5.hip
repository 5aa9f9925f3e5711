// Operator-emission kernels of dimension 5 (see kernels.h).
#include "kernels.h"

namespace pcms {
PCMS_DEFINE_DIM_OPERATOR(5)
}  // namespace pcms
