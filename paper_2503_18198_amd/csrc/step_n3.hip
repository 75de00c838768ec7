// Step kernels (hot-steps copies) for 3-mode tensors (2 input modes per nonzero).
#include "step_kernel.h"

namespace mk {
template hipError_t launch_step_nin<2>(const DevMode&, int, int, const void* const*, const uint32_t* const*,
                                        uint32_t, float*, float*, const Geometry&, uint32_t, hipStream_t);
}  // namespace mk
