// Gather-probe kernels for 5- to 8-mode tensors.
#include "probe_kernel.h"

namespace mk {
namespace part {
template hipError_t launch_probe_nin<4>(const DevMode&, int, int, const void* const*, float*, const Geometry&, int,
                                        hipStream_t);
template hipError_t launch_probe_nin<5>(const DevMode&, int, int, const void* const*, float*, const Geometry&, int,
                                        hipStream_t);
template hipError_t launch_probe_nin<6>(const DevMode&, int, int, const void* const*, float*, const Geometry&, int,
                                        hipStream_t);
template hipError_t launch_probe_nin<7>(const DevMode&, int, int, const void* const*, float*, const Geometry&, int,
                                        hipStream_t);
}  // namespace part
}  // namespace mk
