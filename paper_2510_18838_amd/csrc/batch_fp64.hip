// Persistent batched-transfer kernel, FP64 variant (see batch_kernel.h).
#include "batch_kernel.h"

namespace pcms {
PCMS_DEFINE_BATCH_KERNEL(PCMS_FP64)
}  // namespace pcms
