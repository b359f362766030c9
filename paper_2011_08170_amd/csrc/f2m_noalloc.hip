// Fixed device workspace of f2m_gdp_step_noalloc: a file-scope device array
// that every context on a device shares, so that entry point needs no
// allocation.  Host code never passes the array's name to a kernel (on the
// host it is only a stand-in symbol); it asks the runtime for the array's
// device address once per device and passes that address instead.
#include "f2m_internal.h"

#include <mutex>
#include <vector>

namespace f2m {

namespace {

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_mu;
std::vector<void *> g_ptr;   // per device: the array's device address, or null

}  // namespace

// The device address of this device's copy of the array; the device must be
// current.  Looked up once per device, then served from the table.
hipError_t noalloc_scratch(int device, void **ptr)
{
    *ptr = nullptr;
    if (device < 0) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_ptr.size() <= device) g_ptr.resize(device + 1, nullptr);
    if (!g_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[device] = p;
    }
    *ptr = g_ptr[device];
    return hipSuccess;
}

}  // namespace f2m
