// The fused step for FP64 storage (plain and shifted).
#include "lbmix_step_kernel.h"

namespace lbmix {
LBMIX_STEP_STORE(double);
}  // namespace lbmix
