// Partition kernels for 6-mode tensors (5 input modes per nonzero).
#include "part_kernel.h"

namespace mk {
template hipError_t launch_part_nin<5>(const DevMode&, int, int, const void* const*, const uint32_t* const*,
                                         uint32_t, float*, float*, const Geometry&, hipStream_t);
}  // namespace mk
