// Step kernels (hot-steps copies) for 4-mode tensors (3 input modes per nonzero).
#include "step_kernel.h"

namespace mk {
template hipError_t launch_step_nin<3>(const DevMode&, int, int, const void* const*, const uint32_t* const*,
                                        uint32_t, float*, float*, const Geometry&, uint32_t, hipStream_t);
}  // namespace mk
