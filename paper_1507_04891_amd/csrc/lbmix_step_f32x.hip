// The fused step for FP32 storage with FP64 arithmetic and stochastically rounded stores.
#include "lbmix_step_kernel.h"

namespace lbmix {
LBMIX_STEP_STORE(F32X);
}  // namespace lbmix
