// The fused step for FP32 storage (plain and shifted).
#include "lbmix_step_kernel.h"

namespace lbmix {
LBMIX_STEP_STORE(float);
}  // namespace lbmix
