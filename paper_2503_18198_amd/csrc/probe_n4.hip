// Gather-probe kernels for 4-mode tensors (3 input modes).
#include "probe_kernel.h"

namespace mk {
namespace part {
template hipError_t launch_probe_nin<3>(const DevMode&, int, int, const void* const*, float*, const Geometry&, int,
                                        hipStream_t);
}  // namespace part
}  // namespace mk
