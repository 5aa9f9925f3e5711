// Persistent batched-transfer kernel, MIXED_REFINE variant (see batch_kernel.h).
#include "batch_kernel.h"

namespace pcms {
PCMS_DEFINE_BATCH_KERNEL(PCMS_MIXED_REFINE)
}  // namespace pcms
