// Library-owned scratch memory for fip_dgemm_noalloc, the entry point for
// callers that cannot allocate device memory (code being captured into a
// graph, tight serving loops, harnesses that forbid allocation).
//
// The array lives in the library's device code object: every GPU the library
// runs on holds its own copy, at its own address, until the process ends.  In
// host code `scratch` is only a stand-in for the symbol; its device address
// comes from hipGetSymbolAddress, looked up once per device with that device
// current, and only that address is ever handed to kernels.
#include <mutex>

#include "fip_internal.h"

namespace fip {
namespace {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

}  // namespace

hipError_t scratch_buffer(void** ptr)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (p == nullptr) return hipErrorInvalidSymbol;
        g_scratch[dev] = p;
    }
    *ptr = g_scratch[dev];
    return hipSuccess;
}

}  // namespace fip
