// Partition kernels of 1024-thread workgroups for the tuned launch shapes of
// 3-mode tensors with fp32 factors (2 or 4 gathers in flight, R = 16, 32, 64).
#include "part_kernel.h"

namespace mk {

template hipError_t launch_part_tuned_wg<1024>(const DevMode&, int, int, const void* const*, float*, float*,
                                             const Geometry&, uint32_t, hipStream_t);
template hipError_t launch_batch_part_tuned_wg<1024>(int, int, const void*, const uint2*, uint32_t, uint32_t,
                                                   hipStream_t);

}  // namespace mk
