// chw_scratch.hip -- the library's static device scratch, used as the
// workspace (the FP32 / int32 / FP64 intermediate between the two HBM passes)
// by chw_forward_noalloc, for callers that cannot allocate device memory.
//
// The array is a file-scope __device__ object: every device the library runs
// on holds its own copy, from the first use on that device until the process
// ends.  Host code never passes the array's name to a kernel or a copy (on the
// host it is only a stand-in for the device object); it asks
// hipGetSymbolAddress once per device, with that device current, and uses the
// address it returns.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "chw_scratch.h"

static __device__ __align__(256) unsigned char scratch[chw::SCRATCH_BYTES];

namespace chw {

namespace {
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;  // device ordinal -> device address of `scratch`
}  // namespace

hipError_t scratch_address(int dev, void **ptr)
{
    *ptr = nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *ptr = it->second;
        return hipSuccess;
    }
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev) return hipErrorInvalidDevice;  // the caller makes `dev` current
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr || (reinterpret_cast<uintptr_t>(p) & 255u)) return hipErrorInvalidSymbol;
    g_scratch_ptr.emplace(dev, p);
    *ptr = p;
    return hipSuccess;
}

}  // namespace chw
