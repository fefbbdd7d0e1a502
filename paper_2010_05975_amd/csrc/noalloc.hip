// Device scratch of the allocation-free solve (cfx_getrs_noalloc): a
// file-scope array in device memory, one copy per GPU the library runs on,
// held until the process ends.  Host code never uses the array's name as an
// address (on the host it is only a stand-in for the symbol): the device
// address is looked up once per device with hipGetSymbolAddress, while that
// device is current, and every later use goes through that address.
#include <mutex>

#include "cfx_internal.h"

namespace cfx {
namespace {

__device__ __align__(256) static char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

}  // namespace

int noalloc_scratch(int device, void **ptr)
{
    if (device < 0 || device >= kMaxDevices) return CFX_ENOTSUP;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[device]) {
        int cur = -1;
        CFX_HIP(hipGetDevice(&cur));
        if (cur != device) return CFX_EHIP;     // called with the device current
        void *p = nullptr;
        CFX_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return CFX_EHIP;
        g_ptr[device] = p;
    }
    *ptr = g_ptr[device];
    return CFX_OK;
}

}  // namespace cfx
