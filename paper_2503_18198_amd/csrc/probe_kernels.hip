// Dispatch of the gather-ceiling probe (mttkrp_gather_probe); the kernels are
// in probe_kernel.h, instantiated per mode count in probe_n*.hip so they
// build in parallel.
#include "probe_kernel.h"

namespace mk {
namespace part {
extern template hipError_t launch_probe_nin<2>(const DevMode&, int, int, const void* const*, float*, const Geometry&,
                                               int, hipStream_t);
extern template hipError_t launch_probe_nin<3>(const DevMode&, int, int, const void* const*, float*, const Geometry&,
                                               int, hipStream_t);
extern template hipError_t launch_probe_nin<4>(const DevMode&, int, int, const void* const*, float*, const Geometry&,
                                               int, hipStream_t);
extern template hipError_t launch_probe_nin<5>(const DevMode&, int, int, const void* const*, float*, const Geometry&,
                                               int, hipStream_t);
extern template hipError_t launch_probe_nin<6>(const DevMode&, int, int, const void* const*, float*, const Geometry&,
                                               int, hipStream_t);
extern template hipError_t launch_probe_nin<7>(const DevMode&, int, int, const void* const*, float*, const Geometry&,
                                               int, hipStream_t);
}  // namespace part

hipError_t launch_gather_probe(const DevMode& m, int R, int dtype, const void* const* fac, float* carry,
                               const Geometry& g, int what, hipStream_t s)
{
    if (m.nnz == 0 || g.nparts == 0) return hipSuccess;
    switch (m.n_in) {
        case 2: return part::launch_probe_nin<2>(m, R, dtype, fac, carry, g, what, s);
        case 3: return part::launch_probe_nin<3>(m, R, dtype, fac, carry, g, what, s);
        case 4: return part::launch_probe_nin<4>(m, R, dtype, fac, carry, g, what, s);
        case 5: return part::launch_probe_nin<5>(m, R, dtype, fac, carry, g, what, s);
        case 6: return part::launch_probe_nin<6>(m, R, dtype, fac, carry, g, what, s);
        case 7: return part::launch_probe_nin<7>(m, R, dtype, fac, carry, g, what, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mk
