// noalloc.hip -- per-GPU scratch of the allocation-free monitor entry point
// (lbm_monitors_async): the per-block partial sums of one monitor reduction
// live in a file-scope device array instead of the caller's work buffer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.hpp"

namespace lbm {

namespace {
// MP_COUNT partial sums for each of at most kScratchBlocks blocks (192 KiB);
// every GPU the library runs on holds its own copy until the process ends.
static __device__ __align__(256) double scratch[kScratchBlocks * MP_COUNT];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};
}  // namespace

// Device address of this GPU's copy of the scratch array, found once per
// device (with that device current) and kept.  In host code the array's
// name is only a stand-in, so kernels are always given this address.
hipError_t scratch_partials(hipStream_t s, double** out)
{
    int dev = 0;
    hipError_t e = hipStreamGetDevice(s, &dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        int cur = 0;
        if ((e = hipGetDevice(&cur)) != hipSuccess) return e;
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        g_ptr[dev] = (double*)p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace lbm
