// Gather-probe kernels for 3-mode tensors (2 input modes).
#include "probe_kernel.h"

namespace mk {
namespace part {
template hipError_t launch_probe_nin<2>(const DevMode&, int, int, const void* const*, float*, const Geometry&, int,
                                        hipStream_t);
}  // namespace part
}  // namespace mk
