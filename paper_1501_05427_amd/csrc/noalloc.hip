// Fixed device scratch for the entry points that must not allocate (gp_kmv_noalloc).
//
// The scratch is one file-scope device array.  Its host-side name is only a stand-in
// for the symbol: host code obtains the array's device address once per device with
// hipGetSymbolAddress (with that device current) and uses that address from then on.
// Every call on a device shares that device's array, so calls that overlap on one device
// race; the array keeps whatever the last call left in it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace gpk {

namespace {

__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch(int device, void** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_addr[device] == nullptr) {
        // the caller has made `device` current: each device holds its own copy of the array
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (p == nullptr) return hipErrorInvalidSymbol;
        g_addr[device] = p;
    }
    *out = g_addr[device];
    return hipSuccess;
}

}  // namespace gpk
