// Persistent batched-transfer kernel, MIXED variant (see batch_kernel.h).
#include "batch_kernel.h"

namespace pcms {
PCMS_DEFINE_BATCH_KERNEL(PCMS_MIXED)
}  // namespace pcms
