// The fused step for BF16 storage (plain and shifted).
#include "lbmix_step_kernel.h"

namespace lbmix {
LBMIX_STEP_STORE(BF16);
}  // namespace lbmix
