// Partition kernels for 3-mode tensors (2 input modes per nonzero).
#include "part_kernel.h"

namespace mk {
template hipError_t launch_part_nin<2>(const DevMode&, int, int, const void* const*, const uint32_t* const*,
                                         uint32_t, float*, float*, const Geometry&, uint32_t, hipStream_t);
template size_t part_desc_bytes_nin<2>();
template void fill_part_desc_nin<2>(void*, const DevMode&, int, int, const void* const*, float*, float*, uint32_t);
template hipError_t launch_batch_part_nin<2>(int, int, const void*, const uint2*, uint32_t, uint32_t, hipStream_t);
}  // namespace mk
