// The fused step for FP16 storage (plain and shifted).
#include "lbmix_step_kernel.h"

namespace lbmix {
LBMIX_STEP_STORE(F16);
}  // namespace lbmix
