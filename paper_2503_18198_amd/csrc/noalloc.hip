// mttkrp_run_noalloc: the per-mode MTTKRP for callers that cannot allocate
// device memory.  The carry rows (partials of output rows cut by partition
// boundaries, added in partition order by the fix-up kernel) live in a
// file-scope device array instead of memory the library allocates.  Host code
// never passes the array's name to a kernel: its device address is looked up
// once per device with hipGetSymbolAddress and kept.
#include <mutex>

#include "internal.h"

namespace {

constexpr uint64_t kScratchBytes = 4ull << 20;   // 8192 partitions x 2 carry rows x 64 fp32
__device__ __align__(256) float scratch[kScratchBytes / sizeof(float)];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
float* g_scratch[kMaxDevices] = {};   // device address of `scratch` on each device, once looked up

// Device address of the current device's copy of `scratch`.
hipError_t scratch_on_current(int* dev_out, float** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = static_cast<float*>(p);
    }
    *dev_out = dev;
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

mttkrp_status mttkrp_run_noalloc(mttkrp_handle h, int mode, const float* const* factors, float* out, int R,
                                 hipStream_t stream)
{
    int dev = -1;
    float* carry = nullptr;
    const hipError_t e = scratch_on_current(&dev, &carry);
    if (e != hipSuccess) return mk::set_error(MTTKRP_EHIP, hipGetErrorString(e));
    return mk::run_fp32_with_carry(h, mode, factors, out, R, dev, carry, kScratchBytes, stream);
}

uint64_t mttkrp_noalloc_scratch_bytes(void) { return kScratchBytes; }

}  // extern "C"
