// noalloc.hip -- the device scratch of the allocation-free entry point.
//
// rbf_matvec_device_noalloc stages the weights and the product in the cell-
// sorted order, as rbf_matvec_device does in the caller's original order, but
// in a fixed array that the code object carries instead of blocks it
// allocates.  Each device that loads the library holds its own copy of the
// array until the process ends; its address on a device comes from
// hipGetSymbolAddress, taken once per device with that device current (the
// array's name in host code is only a host-side stand-in).
#include <hip/hip_runtime.h>

#include <mutex>

#include "rbf_internal.hpp"

namespace {

// two vectors of kNoAllocMaxPoints doubles: the sorted weights, the sorted product
static __device__ __align__(256) double scratch[2 * rbf::kNoAllocMaxPoints];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

namespace rbf {

hipError_t noalloc_scratch(int device, double** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[device] = p;
    }
    *out = static_cast<double*>(g_ptr[device]);
    return hipSuccess;
}

}  // namespace rbf
