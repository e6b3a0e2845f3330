// Device-side storage of the allocation-free stepping entry point
// (fe_advance_noalloc): the job table of the step launches lives in a
// file-scope device array instead of a caller workspace.
//
// In host code the array's name is only a stand-in for the symbol, not a
// device address.  fe_create resolves the array's address on its device
// (with that device current) once per device through hipGetSymbolAddress;
// every later use goes through that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fe_internal.h"

namespace {

__device__ __align__(256) unsigned char scratch[fe::kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};

}  // namespace

namespace fe {

hipError_t noalloc_setup(int device)
{
    // devices beyond the table keep no address: fe_advance_noalloc reports
    // FE_ERR_DEVICE there, every other entry point works
    if (device < 0 || device >= kMaxDevices) return hipSuccess;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_addr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;   // the caller makes it current
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_addr[device] = p;
    return hipSuccess;
}

void *noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_addr[device];
}

}  // namespace fe
