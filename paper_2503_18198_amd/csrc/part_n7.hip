// Partition kernels for 7-mode tensors (6 input modes per nonzero).
#include "part_kernel.h"

namespace mk {
template hipError_t launch_part_nin<6>(const DevMode&, int, int, const void* const*, const uint32_t* const*,
                                         uint32_t, float*, float*, const Geometry&, hipStream_t);
}  // namespace mk
